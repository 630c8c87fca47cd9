// Cone pass: one traversal per pulse, shared by all of its subrays.
//
// Every subray of a pulse leaves the origin O within the largest subray angle
// a_max of the beam axis d (Sec. 3.4, Fig. 6).  Written with the axial distance t
// as parameter, a subray point is O + t d + w with |w| <= t tan(a_max), so every
// coordinate stays within t k of the axis point (k = tan a_max plus rounding
// slack).  A node box can therefore hold a subray hit only if, for some t >= 0
// and every axis a,  O_a + t (d_a + k) >= lo_a  and  O_a + t (d_a - k) <= hi_a:
// a slab test whose two planes move with different slopes.  One lane per pulse
// walks the LBVH with that test (near child first, FP32 with the same per-ray
// padding as the subray traversal) and records every leaf it reaches; the
// subrays then test only those triangles, in FP64 as before, so the result is
// the same closest hit a per-subray traversal finds.
//
// Culling: when the four corner rays of a square pyramid around the cone all hit
// one triangle strictly inside it, every subray (its direction lies inside that
// pyramid) hits that triangle, at an axial distance no larger than the largest
// corner distance; nodes that start beyond it cannot hold a closest hit.
// A pulse with more than kCandMax (255) candidates is marked for full per-subray
// traversal.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "device_common.h"
#include "vls_internal.h"

namespace vls {
namespace {

struct Cone {
    double O[3];
    // axis and the pyramid's half-width vectors (1 + 1e-3) tan(a_max) u, v in
    // FP32: the widening (2.5e-7 rad at the largest beams here) covers the FP32
    // rounding of the corner directions (~1e-7 rad), so the pyramid of the
    // rounded corners still contains every subray
    float D[3];
    float U[3];
    float V[3];
    float i1[3], i2[3], c1[3], c2[3];
    bool mixed;      // some axis has d_a - k < 0 < d_a + k
    int mixed_axes;  // bit a set for each such axis
};

// The pulse's cone from its basis (the subrays' own basis, computed the same
// way; see pulse_basis).
__device__ __forceinline__ bool setup_cone(const double* __restrict__ o, const dev::Basis& B, double tana,
                                           float scene_mag, Cone& c)
{
#pragma clang fp contract(off)
    const double* n = B.n;
    const double a = B.a, b = B.b;
    double sgn = copysign(1.0, n[2]);
    double u[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    double v[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    double omax = 0.0;
    const double w = tana * (1.0 + 1e-3);
    for (int i = 0; i < 3; ++i) {
        c.O[i] = o[i];
        c.D[i] = (float)n[i];
        c.U[i] = (float)(w * u[i]);
        c.V[i] = (float)(w * v[i]);
        omax = fmax(omax, fabs(o[i]));
    }
    if (!(omax < INFINITY)) return false;
    double pad = (omax + (double)scene_mag + 1.0) * 1.9073486328125e-06;  // 2^-19, as for subrays
    // slope: tan(a_max), the FP32 rounding of the axis (~2^-23 rad) and slack
    float k = (float)(tana * (1.0 + 1e-6) + 4e-7);
    c.mixed = false;
    c.mixed_axes = 0;
    for (int i = 0; i < 3; ++i) {
        float da = (float)n[i];
        float s1 = da + k, s2 = da - k;
        if (s1 == 0.0f) s1 = 1e-30f;
        if (s2 == 0.0f) s2 = -1e-30f;
        if (s1 > 0.0f && s2 < 0.0f) {
            c.mixed = true;
            c.mixed_axes |= 1 << i;
        }
        c.i1[i] = 1.0f / s1;
        c.i2[i] = 1.0f / s2;
        c.c1[i] = (float)(c.O[i] + pad) * c.i1[i];
        c.c2[i] = (float)(c.O[i] - pad) * c.i2[i];
    }
    return true;
}

// Interval of axial distances over which the cone can lie inside the slab
// [lo, hi] of one axis.  tA is where the side of slope d + k crosses lo, tB where
// the side of slope d - k crosses hi.  When both slopes have one sign, the
// interval is [tA, tB] (positive) or [tB, tA] (negative); an ordering the other
// way round only occurs for an interval that ends before t = 0, which the caller
// rejects anyway, so min and max give it.  MIXED (slopes of both signs): the
// interval is [max(tA, tB), inf).
template <bool MIXED>
__device__ __forceinline__ void cone_axis(const Cone& c, int a, float lo, float hi, float& lower, float& upper)
{
    const float tA = fmaf(lo, c.i1[a], -c.c1[a]);
    const float tB = fmaf(hi, c.i2[a], -c.c2[a]);
    if (!MIXED) {
        lower = fminf(tA, tB);
        upper = fmaxf(tA, tB);
    } else {
        const bool p1 = c.i1[a] > 0.0f, p2 = c.i2[a] > 0.0f;
        const float mn = fminf(tA, tB), mx = fmaxf(tA, tB);
        lower = (p1 && !p2) ? mx : mn;
        upper = (p1 && !p2) ? INFINITY : mx;
    }
}

// MA: the axes (bit a for axis a) that take the mixed-sign form; it must
// include every mixed axis of every lane that uses it (the form is also right
// for an axis whose slopes have one sign, only dearer).
template <int MA>
__device__ __forceinline__ bool cone_box(const Cone& c, float lx, float ly, float lz, float hx, float hy, float hz,
                                         float tcull, float& tn)
{
    float l0, u0, l1, u1, l2, u2;
    cone_axis<(MA & 1) != 0>(c, 0, lx, hx, l0, u0);
    cone_axis<(MA & 2) != 0>(c, 1, ly, hy, l1, u1);
    cone_axis<(MA & 4) != 0>(c, 2, lz, hz, l2, u2);
    float n0 = fmaxf(fmaxf(l0, l1), fmaxf(l2, 0.0f));
    float f0 = fminf(fminf(u0, u1), fminf(u2, tcull));
    tn = n0;
    return n0 <= f0;
}

// Largest axial distance at which the whole pyramid around the cone meets the
// triangle (an upper bound), or +inf if some corner ray may miss it.  Each
// corner ray O + t d, d = D +- U +- V, must hit the triangle strictly inside
// all three edges (Moller-Trumbore; a sufficient condition only: a miss just
// means no cull).  With s = O - a, n = e1 x e2, w = e2 x s and q = s x e1, the
// unnormalised determinant and barycentrics are triple products:
// det = -d . n, u det = d . w, v det = d . q, t det = e2 . q, so each corner
// costs three dot products.  In FP32: e1, e2 and s are rounded once (s from
// FP64), a cross product by fused multiply-adds and a dot product with the
// exact corner direction err by less than 8 u |x|1 |y|1 |z|1 for the triple
// product of x, y, z (u = 2^-24); each test is taken with twice that bound
// against it, so a pass holds in exact arithmetic, and the distance is the
// bound's largest quotient rounded up.
__device__ __forceinline__ float cover_distance(const Cone& c, const float4* __restrict__ tris, int li)
{
    const float4 A = tris[3 * li], B = tris[3 * li + 1], C = tris[3 * li + 2];
    const float e1[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
    const float e2[3] = {C.x - A.x, C.y - A.y, C.z - A.z};
    const float s3[3] = {(float)(c.O[0] - A.x), (float)(c.O[1] - A.y), (float)(c.O[2] - A.z)};
    const float q[3] = {fmaf(s3[1], e1[2], -(s3[2] * e1[1])), fmaf(s3[2], e1[0], -(s3[0] * e1[2])),
                        fmaf(s3[0], e1[1], -(s3[1] * e1[0]))};
    const float w[3] = {fmaf(e2[1], s3[2], -(e2[2] * s3[1])), fmaf(e2[2], s3[0], -(e2[0] * s3[2])),
                        fmaf(e2[0], s3[1], -(e2[1] * s3[0]))};
    const float nv[3] = {fmaf(e1[1], e2[2], -(e1[2] * e2[1])), fmaf(e1[2], e2[0], -(e1[0] * e2[2])),
                         fmaf(e1[0], e2[1], -(e1[1] * e2[0]))};
    const float tn = fmaf(e2[0], q[0], fmaf(e2[1], q[1], e2[2] * q[2]));
    const float l1 = fabsf(e1[0]) + fabsf(e1[1]) + fabsf(e1[2]);
    const float l2 = fabsf(e2[0]) + fabsf(e2[1]) + fabsf(e2[2]);
    const float ls = fabsf(s3[0]) + fabsf(s3[1]) + fabsf(s3[2]);
    // |d|1 of every corner is at most |D|1 + |U|1 + |V|1
    const float dl = (fabsf(c.D[0]) + fabsf(c.D[1]) + fabsf(c.D[2])) + (fabsf(c.U[0]) + fabsf(c.U[1]) + fabsf(c.U[2])) +
                     (fabsf(c.V[0]) + fabsf(c.V[1]) + fabsf(c.V[2]));
    const float Ed = 0x1p-20f * dl * l1 * l2, Eu = 0x1p-20f * dl * l2 * ls, Ev = 0x1p-20f * dl * ls * l1;
    const float Et = 0x1p-20f * l2 * ls * l1;
    // beyond FP32's comfortable range (or not finite): no cull
    if (!(Ed + Eu + Ev + Et < 1e30f)) return INFINITY;
    float dmin = INFINITY;  // smallest determinant bound over the corners
    for (int k = 0; k < 4; ++k) {
        const float su = (k & 1) ? 1.0f : -1.0f, sv = (k & 2) ? 1.0f : -1.0f;
        const float d[3] = {fmaf(sv, c.V[0], fmaf(su, c.U[0], c.D[0])), fmaf(sv, c.V[1], fmaf(su, c.U[1], c.D[1])),
                            fmaf(sv, c.V[2], fmaf(su, c.U[2], c.D[2]))};
        float det = -fmaf(d[0], nv[0], fmaf(d[1], nv[1], d[2] * nv[2]));
        float un = fmaf(d[0], w[0], fmaf(d[1], w[1], d[2] * w[2]));
        float vn = fmaf(d[0], q[0], fmaf(d[1], q[1], d[2] * q[2]));
        float t = tn;
        if (det < 0.0f) {  // same tests with det > 0
            det = -det;
            un = -un;
            vn = -vn;
            t = -t;
        }
        const float dlo = det - Ed;
        if (!(dlo > 0.0f && un > Eu && vn > Ev && (un + vn) * (1.0f + 0x1p-22f) + (Eu + Ev) < dlo && t > Et))
            return INFINITY;
        dmin = fminf(dmin, dlo);
    }
    return (fabsf(tn) + Et) / dmin * (1.0f + 0x1p-20f);
}

// A stack entry of the cone walk: the node and, with cover tests, its entry
// distance (an entry pushed before a cull distance was known is dropped when
// popped beyond it).  Without cover tests the cull distance stays infinite, so
// the node alone is kept: half the LDS per entry, more wavefronts per CU.
template <bool COVER>
struct ConeEnt;
template <>
struct ConeEnt<true> {
    using T = int2;
    static __device__ __forceinline__ T make(int node, float t) { return make_int2(node, __float_as_int(t)); }
    static __device__ __forceinline__ T none() { return make_int2(-1, 0); }
    static __device__ __forceinline__ int node(T e) { return e.x; }
    static __device__ __forceinline__ bool live(T e, float tcull) { return __int_as_float(e.y) <= tcull; }
};
template <>
struct ConeEnt<false> {
    using T = int;
    static __device__ __forceinline__ T make(int node, float) { return node; }
    static __device__ __forceinline__ T none() { return -1; }
    static __device__ __forceinline__ int node(T e) { return e; }
    static __device__ __forceinline__ bool live(T, float) { return true; }
};

// One lane's cone traversal: writes the candidate leaves to out[e0..] and
// returns their count (-1: more than cap, or a corrupted structure).  out is
// 16-byte aligned; entries below e0 (a row's count) are left to the caller.
//
// A leaf is recorded and the walk moves on at once; the cover test (the
// expensive part, and only an aid to culling) runs on a lane's first untested
// leaf in batches, when a quarter of the wavefront's walking lanes (or 16) have
// one waiting, so that the wavefront does not pay for it in every step in which
// some lane sits at a leaf.  A later or skipped cover test only culls less; the
// list still holds every leaf the cone reaches before the cull that applies.
template <bool COUNT, int MA, bool COVER = true>
__device__ __forceinline__ int cone_walk(const SceneDev& scene, const Cone& c, int* __restrict__ out, int e0, int cap,
                                         typename ConeEnt<COVER>::T* my, int ring_mask, int& visits)
{
    int n = 0;
    int b0 = 0, b1 = 0, b2 = 0, b3 = 0;  // the row's current group of four entries
    float tcull = INFINITY;
    const int stride = blockDim.x;
    // stack entries carry their entry distance, so nodes pushed before a cull
    // distance was known are dropped when popped
    using E = ConeEnt<COVER>;
    typename E::T spill[kMaxSpill];
    int sp = 0, nlow = 0;
    int node = scene.root;
    const int n_int = scene.n_tri - 1;
    int budget = 2 * scene.n_tri + 64;
    bool busy = true;
    int pend = -1;  // first recorded leaf not yet cover-tested
    while (true) {
        if (busy) {
            bool pop = false;
            if (--budget <= 0 || node >= n_int || ~node >= scene.n_tri) {
                n = -1;
                busy = false;
            } else if (node >= 0) {
                // a four-wide record: the node's grandchildren (or leaf children)
                if (COUNT) ++visits;
                const float4* nd = scene.nodes4 + 8 * node;
                const float4 LX = nd[0], LY = nd[1], LZ = nd[2], HX = nd[3], HY = nd[4], HZ = nd[5], RF = nd[6];
                float t[4];
                int r[4] = {__float_as_int(RF.x), __float_as_int(RF.y), __float_as_int(RF.z), __float_as_int(RF.w)};
                t[0] = cone_box<MA>(c, LX.x, LY.x, LZ.x, HX.x, HY.x, HZ.x, tcull, t[0]) && r[0] != kEmpty4 ? t[0] : INFINITY;
                t[1] = cone_box<MA>(c, LX.y, LY.y, LZ.y, HX.y, HY.y, HZ.y, tcull, t[1]) && r[1] != kEmpty4 ? t[1] : INFINITY;
                t[2] = cone_box<MA>(c, LX.z, LY.z, LZ.z, HX.z, HY.z, HZ.z, tcull, t[2]) && r[2] != kEmpty4 ? t[2] : INFINITY;
                t[3] = cone_box<MA>(c, LX.w, LY.w, LZ.w, HX.w, HY.w, HZ.w, tcull, t[3]) && r[3] != kEmpty4 ? t[3] : INFINITY;
                // nearest first: sort the four (distance, ref) pairs, misses (inf) last
#define VLS_CX(a, b)                                  \
    if (t[b] < t[a]) {                                \
        const float tt = t[a]; t[a] = t[b]; t[b] = tt; \
        const int rr = r[a]; r[a] = r[b]; r[b] = rr;   \
    }
                VLS_CX(0, 1) VLS_CX(2, 3) VLS_CX(0, 2) VLS_CX(1, 3) VLS_CX(1, 2)
#undef VLS_CX
                node = r[0];
                pop = !(t[0] < INFINITY);
                // the others are pushed farthest first, so the nearer ones pop first
                for (int q = 3; q >= 1; --q) {
                    if (t[q] < INFINITY) {
                        if (sp - nlow > ring_mask) {
                            if (nlow < kMaxSpill) spill[nlow] = my[(nlow & ring_mask) * stride];
                            ++nlow;
                        }
                        my[(sp & ring_mask) * stride] = E::make(r[q], t[q]);
                        ++sp;
                    }
                }
            } else if (n == cap) {  // too many: a longer list or the subrays' own walks
                n = -1;
                busy = false;
            } else {
                // entry e0 + n goes to the lane's four-entry buffer; a full,
                // 16-byte aligned group of four is stored at once (a row's
                // entry 0, the count, is stored after the walk)
                const int e = e0 + n, id = ~node;
                b0 = (e & 3) == 0 ? id : b0;
                b1 = (e & 3) == 1 ? id : b1;
                b2 = (e & 3) == 2 ? id : b2;
                b3 = (e & 3) == 3 ? id : b3;
                if ((e & 3) == 3) *reinterpret_cast<int4*>(out + (e - 3)) = make_int4(b0, b1, b2, b3);
                ++n;
                if (COVER && pend < 0) pend = ~node;
                pop = true;
            }
            if (pop) {
                // pop the next node that can still hold a closest hit
                busy = false;
                while (sp > 0) {
                    --sp;
                    typename E::T e;
                    if (sp < nlow) {
                        e = sp < kMaxSpill ? spill[sp] : E::none();
                        nlow = sp;
                    } else {
                        e = my[(sp & ring_mask) * stride];
                    }
                    if (E::live(e, tcull)) {
                        node = E::node(e);
                        busy = true;
                        break;
                    }
                }
            }
        }
        const unsigned long long walking = __ballot(busy);
        if (walking == 0) break;
        const unsigned long long waiting = __ballot(busy && pend >= 0);
        const int nw = __popcll(waiting);
        if (nw >= 16 || 4 * nw >= __popcll(walking)) {
            if (busy && pend >= 0) {
                const float tc = cover_distance(c, scene.tris, pend);
                if (tc < INFINITY) tcull = fminf(tcull, tc);
                pend = -1;
            }
        }
    }
    // the last, partial group: entries (e0 + n) & ~3 .. e0 + n - 1, those below
    // e0 excepted
    if (n > 0) {
        const int e = (e0 + n) & ~3, r = (e0 + n) & 3;
        if (r > 0 && e >= e0) out[e] = b0;
        if (r > 1 && e + 1 >= e0) out[e + 1] = b1;
        if (r > 2 && e + 2 >= e0) out[e + 2] = b2;
    }
    return n;
}

// COVER: run the cover tests (see cone_walk).
template <bool COUNT, bool COVER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_cone(SceneDev scene, double tana, PulsesDev pulses, int* __restrict__ cand,
                                              long long first, long long count, int ring_mask,
                                              unsigned long long* counts, int* ovf_list, unsigned long long* ovf_ctr,
                                              double* basis_out, int cap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < count;
    const long long p = first + i;
    int visits = 0;
    Cone c;
    dev::Basis B;
    const bool bok = active && dev::pulse_basis(pulses.dirs + 3 * p, B);
    if (basis_out && active) {
        // the pulse's basis for the fused kernel (n_x NaN: no valid direction)
        double* w = basis_out + 5 * p;
        w[0] = bok ? B.n[0] : (double)NAN;
        w[1] = bok ? B.n[1] : 0.0;
        w[2] = bok ? B.n[2] : 0.0;
        w[3] = bok ? B.a : 0.0;
        w[4] = bok ? B.b : 0.0;
    }
    const bool ok = bok && scene.n_tri > 0 && setup_cone(pulses.origins + 3 * p, B, tana, scene.bounds[12], c);
    int n = 0;
    int* out = cand + p * (kCandMax + 1);
    auto* my = reinterpret_cast<typename ConeEnt<COVER>::T*>(smem) + threadIdx.x;
    // the cheaper slab test serves every axis no lane of the wavefront has with
    // slopes of both signs: none, only x or only y (scan lines along an axis),
    // else all three take the mixed form
    const unsigned long long mx = __ballot(ok && (c.mixed_axes & 1)), my_ = __ballot(ok && (c.mixed_axes & 2)),
                             mz = __ballot(ok && (c.mixed_axes & 4));
    if ((mx | my_ | mz) == 0) {
        if (ok) n = cone_walk<COUNT, 0, COVER>(scene, c, out, 1, cap, my, ring_mask, visits);
    } else if ((my_ | mz) == 0) {
        if (ok) n = cone_walk<COUNT, 1, COVER>(scene, c, out, 1, cap, my, ring_mask, visits);
    } else if ((mx | mz) == 0) {
        if (ok) n = cone_walk<COUNT, 2, COVER>(scene, c, out, 1, cap, my, ring_mask, visits);
    } else {
        if (ok) n = cone_walk<COUNT, 7, COVER>(scene, c, out, 1, cap, my, ring_mask, visits);
    }
    if (active) out[0] = n;
    if (ovf_list) {
        // overflowed pulses go to the list, one counter update per wavefront
        const unsigned long long m = __ballot(active && n < 0);
        if (m) {
            const int lane = threadIdx.x & (kWave - 1);
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(ovf_ctr, (unsigned long long)__popcll(m));
            const unsigned b_lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, leader);
            const unsigned b_hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(base >> 32), leader);
            const unsigned long long b = ((unsigned long long)b_hi << 32) | b_lo;
            if (active && n < 0) ovf_list[b + dev::lanes_below(m)] = (int)i;
        }
    }
    if (COUNT) {
        unsigned long long v = (unsigned long long)visits;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(counts + 1, v);
    }
}

// Second pass over the overflowed pulses: list[i] (i < *ctr) is a pulse index
// relative to the launch.  Pulse i of the list walks again with room for
// kLongMax candidates in long row i (while i < rows); a list that fits makes
// the pulse's row (count, long row index); the others go to list2 for the packet
// walk, one counter update per wavefront.  A grid-stride loop covers the list.
// COVER: cover tests as in the first pass.  The long pass runs without them:
// pulses that overflow are the ones no triangle covers (a canopy's leaves), so
// the tests would only cost time (8.1 against 8.9 ms for both passes on the
// vegetation workload, the same lists' worth of fused time).
template <bool COVER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_cone_long(
    SceneDev scene, double tana, PulsesDev pulses, int* __restrict__ cand, const int* __restrict__ list,
    const unsigned long long* ctr, long long rows, int* __restrict__ long_rows, int* list2,
    unsigned long long* ctr2, int ring_mask)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long n_ovf = (long long)__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long stride = (long long)gridDim.x * blockDim.x;
    auto* my = reinterpret_cast<typename ConeEnt<COVER>::T*>(smem) + threadIdx.x;
    const long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // every lane of a wavefront takes the same number of turns (the ballot
    // below needs the whole wavefront)
    const long long wave0 = start - (threadIdx.x & (kWave - 1));
    for (long long base = wave0; base < n_ovf; base += stride) {
        const long long i = base + (threadIdx.x & (kWave - 1));
        const bool active = i < n_ovf;
        const long long q = active ? list[i] : 0;
        int n = -1;
        if (active && i < rows) {
            dev::Basis B;
            Cone c;
            const bool ok = scene.n_tri > 0 && dev::load_basis(pulses.basis + 5 * q, B) &&
                            setup_cone(pulses.origins + 3 * q, B, tana, scene.bounds[12], c);
            int visits = 0;
            int* out = long_rows + (size_t)i * kLongMax;
            // the slab test's form by the wavefront's mixed-sign axes, as in k_cone
            const unsigned long long mx = __ballot(ok && (c.mixed_axes & 1)),
                                     my_ = __ballot(ok && (c.mixed_axes & 2)), mz = __ballot(ok && (c.mixed_axes & 4));
            if ((mx | my_ | mz) == 0) {
                if (ok) n = cone_walk<false, 0, COVER>(scene, c, out, 0, kLongMax, my, ring_mask, visits);
            } else if ((my_ | mz) == 0) {
                if (ok) n = cone_walk<false, 1, COVER>(scene, c, out, 0, kLongMax, my, ring_mask, visits);
            } else if ((mx | mz) == 0) {
                if (ok) n = cone_walk<false, 2, COVER>(scene, c, out, 0, kLongMax, my, ring_mask, visits);
            } else {
                if (ok) n = cone_walk<false, 7, COVER>(scene, c, out, 0, kLongMax, my, ring_mask, visits);
            }
            if (n > kCandMax) {
                int* row = cand + q * (kCandMax + 1);
                row[0] = n;
                row[1] = (int)i;
            } else if (n >= 0) {
                // the second walk's culls came at other times and it fits a row
                int* row = cand + q * (kCandMax + 1);
                for (int j = 0; j < n; ++j) row[1 + j] = out[j];
                row[0] = n;
            }
        }
        const unsigned long long m = __ballot(active && n < 0);
        if (m) {
            const int lane = threadIdx.x & (kWave - 1);
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long b = 0;
            if (lane == leader) b = atomicAdd(ctr2, (unsigned long long)__popcll(m));
            const unsigned b_lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, leader);
            const unsigned b_hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), leader);
            const unsigned long long bb = ((unsigned long long)b_hi << 32) | b_lo;
            if (active && n < 0) list2[bb + dev::lanes_below(m)] = (int)q;
        }
    }
}

__global__ __launch_bounds__(256) void k_leaf_to_orig(const int32_t* __restrict__ leaf_tri, int* __restrict__ cand,
                                                      long long n)
{
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int* c = cand + p * (kCandMax + 1);
    int cnt = c[0];
    for (int i = 0; i < cnt && i < kCandMax; ++i) c[1 + i] = leaf_tri[c[1 + i]];
}

}  // namespace

hipError_t launch_leaf_to_orig(const int32_t* leaf_tri, int* cand, long long n_pulses, hipStream_t stream)
{
    hipLaunchKernelGGL(k_leaf_to_orig, dim3((unsigned)((n_pulses + 255) / 256)), dim3(256), 0, stream, leaf_tri, cand,
                       n_pulses);
    return hipGetLastError();
}

hipError_t launch_cone_long(const SceneDev& scene, double tan_max, const PulsesDev& pulses, int* cand,
                            const int* list, const unsigned long long* ctr, long long n, int* longw,
                            const LaunchCfg& cfg, hipStream_t stream)
{
    int* list2 = long_ws_list(longw, n);
    unsigned long long* ctr2 = long_ws_ctr(longw, n);
    hipError_t e = launch_fill_u64(ctr2, 2, 0ull, stream);
    if (e != hipSuccess) return e;
    if (n <= 0) return hipSuccess;
    // one lane per long row at most; the list's count is read on the device
    const int block = kWave;
    const long long rows = long_rows(n);
    const unsigned grid = (unsigned)((rows + block - 1) / block);
    const size_t lds = sizeof(ConeEnt<false>::T) * (size_t)kConeRing * block;
    (void)cfg;
    hipLaunchKernelGGL(k_cone_long<false>, dim3(grid), dim3(block), lds, stream, scene, tan_max, pulses, cand, list,
                       ctr, rows, longw, list2, ctr2, kConeRing - 1);
    return hipGetLastError();
}

hipError_t launch_cone(const SceneDev& scene, double tan_max, const PulsesDev& pulses, int* cand, long long first,
                       long long count, const LaunchCfg& cfg, unsigned long long* counts, int* ovf_list,
                       unsigned long long* ovf_ctr, double* basis_out, hipStream_t stream, int cap, bool cover)
{
    if (ovf_list) {
        hipError_t e = launch_fill_u64(ovf_ctr, 2, 0ull, stream);
        if (e != hipSuccess) return e;
    }
    if (count <= 0) return hipSuccess;
    const int block = 64 * cfg.block_waves;
    unsigned grid = (unsigned)((count + block - 1) / block);
    // the cone pass keeps its own ring depth: a four-wide visit can push three
    // entries.  With cover tests the walks stop behind covering triangles and
    // stay shallow, and 8 entries per lane leave LDS for more wavefronts (ALS
    // workload 0.72 -> 0.69 ms); without them (deep canopy walks) 8 entries
    // spill to scratch too often (vegetation 5.5 -> 6.0 ms), so they keep 16
    const int ring = cover ? kConeRingCover : kConeRing;
    size_t lds = (cover ? sizeof(ConeEnt<true>::T) : sizeof(ConeEnt<false>::T)) * (size_t)ring * block;
    int mask = ring - 1;
#define VLS_CONE_LAUNCH(COUNT, COVER)                                                                          \
    hipLaunchKernelGGL((k_cone<COUNT, COVER>), dim3(grid), dim3(block), lds, stream, scene, tan_max, pulses, cand, \
                       first, count, mask, counts, ovf_list, ovf_ctr, basis_out, cap)
    if (counts) {
        if (cover) VLS_CONE_LAUNCH(true, true);
        else VLS_CONE_LAUNCH(true, false);
    } else {
        if (cover) VLS_CONE_LAUNCH(false, true);
        else VLS_CONE_LAUNCH(false, false);
    }
#undef VLS_CONE_LAUNCH
    return hipGetLastError();
}

}  // namespace vls
