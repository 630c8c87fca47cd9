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
// A pulse with more than kCandMax (63) candidates is marked for full per-subray
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
    double D[3];
    double U[3];  // tan(a_max) u
    double V[3];  // tan(a_max) v
    float i1[3], i2[3], c1[3], c2[3];
    unsigned pos;  // bit a: d_a + k > 0; bit 3 + a: d_a - k > 0
};

__device__ __forceinline__ bool setup_cone(const double* __restrict__ o, const float* __restrict__ d32, double tana,
                                           float scene_mag, Cone& c)
{
#pragma clang fp contract(off)
    double dx = d32[0], dy = d32[1], dz = d32[2];
    double len = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(len > 0.0) || !(len < INFINITY)) return false;
    double n[3] = {dx / len, dy / len, dz / len};
    double sgn = copysign(1.0, n[2]);
    double a = -1.0 / (sgn + n[2]);
    double b = n[0] * n[1] * a;
    double u[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    double v[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    double omax = 0.0;
    for (int i = 0; i < 3; ++i) {
        c.O[i] = o[i];
        c.D[i] = n[i];
        c.U[i] = tana * u[i];
        c.V[i] = tana * v[i];
        omax = fmax(omax, fabs(o[i]));
    }
    if (!(omax < INFINITY)) return false;
    double pad = (omax + (double)scene_mag + 1.0) * 1.9073486328125e-06;  // 2^-19, as for subrays
    // slope: tan(a_max), the FP32 rounding of the axis (~2^-23 rad) and slack
    float k = (float)(tana * (1.0 + 1e-6) + 4e-7);
    c.pos = 0;
    for (int i = 0; i < 3; ++i) {
        float da = (float)n[i];
        float s1 = da + k, s2 = da - k;
        if (s1 == 0.0f) s1 = 1e-30f;
        if (s2 == 0.0f) s2 = -1e-30f;
        if (s1 > 0.0f) c.pos |= 1u << i;
        if (s2 > 0.0f) c.pos |= 8u << i;
        c.i1[i] = 1.0f / s1;
        c.i2[i] = 1.0f / s2;
        c.c1[i] = (float)(c.O[i] + pad) * c.i1[i];
        c.c2[i] = (float)(c.O[i] - pad) * c.i2[i];
    }
    return true;
}

__device__ __forceinline__ void cone_axis(const Cone& c, int a, float lo, float hi, float& lower, float& upper)
{
    float tA = fmaf(lo, c.i1[a], -c.c1[a]);  // lower plane, slope d_a + k
    float tB = fmaf(hi, c.i2[a], -c.c2[a]);  // upper plane, slope d_a - k
    bool p1 = (c.pos >> a) & 1u, p2 = (c.pos >> (3 + a)) & 1u;
    lower = p1 ? (p2 ? tA : fmaxf(tA, tB)) : tB;
    upper = p2 ? tB : (p1 ? INFINITY : tA);
}

__device__ __forceinline__ bool cone_box(const Cone& c, float lx, float ly, float lz, float hx, float hy, float hz,
                                         float tcull, float& tn)
{
    float l0, u0, l1, u1, l2, u2;
    cone_axis(c, 0, lx, hx, l0, u0);
    cone_axis(c, 1, ly, hy, l1, u1);
    cone_axis(c, 2, lz, hz, l2, u2);
    float n0 = fmaxf(fmaxf(l0, l1), fmaxf(l2, 0.0f));
    float f0 = fminf(fminf(u0, u1), fminf(u2, tcull));
    tn = n0;
    return n0 <= f0;
}

// Moller-Trumbore in FP64 for one corner ray, requiring a margin inside all
// three edges (a sufficient condition only: a miss here just means no cull).
__device__ __forceinline__ bool corner_inside(const double O[3], const double d[3], const double a[3],
                                              const double e1[3], const double e2[3], double& t)
{
    double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    double s[3] = {O[0] - a[0], O[1] - a[1], O[2] - a[2]};
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
    double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    const double m = 1e-9;
    return u > m && v > m && u + v < 1.0 - m && t > 0.0;
}

// Largest axial distance at which the whole pyramid around the cone meets the
// triangle, or +inf if some corner ray misses it.
__device__ __forceinline__ double cover_distance(const Cone& c, const float4* __restrict__ tris, int li)
{
    float4 A = tris[3 * li], B = tris[3 * li + 1], C = tris[3 * li + 2];
    double a[3] = {A.x, A.y, A.z};
    double e1[3] = {(double)B.x - A.x, (double)B.y - A.y, (double)B.z - A.z};
    double e2[3] = {(double)C.x - A.x, (double)C.y - A.y, (double)C.z - A.z};
    double tmax = 0.0;
    for (int q = 0; q < 4; ++q) {
        double su = (q & 1) ? 1.0 : -1.0, sv = (q & 2) ? 1.0 : -1.0;
        double d[3] = {c.D[0] + su * c.U[0] + sv * c.V[0], c.D[1] + su * c.U[1] + sv * c.V[1],
                       c.D[2] + su * c.U[2] + sv * c.V[2]};
        double t;
        if (!corner_inside(c.O, d, a, e1, e2, t)) return INFINITY;
        tmax = fmax(tmax, t);
    }
    return tmax * (1.0 + 1e-9) + 1e-9;
}

template <bool COUNT>
__global__ __launch_bounds__(256) void k_cone(SceneDev scene, double tana, PulsesDev pulses, int* __restrict__ cand,
                                              long long first, long long count, int ring_mask,
                                              unsigned long long* counts)
{
    extern __shared__ __align__(16) unsigned char smem[];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < count;
    const long long p = first + i;
    int visits = 0;
    if (active) {
        int* out = cand + p * (kCandMax + 1);
        int n = 0;
        Cone c;
        if (scene.n_tri > 0 && setup_cone(pulses.origins + 3 * p, pulses.dirs + 3 * p, tana, scene.bounds[12], c)) {
            float tcull = INFINITY;
            const int stride = blockDim.x;
            // stack entries carry their entry distance, so nodes pushed before a
            // cull distance was known are dropped when popped
            int2* my = reinterpret_cast<int2*>(smem) + threadIdx.x;
            int2 spill[kMaxSpill];
            int sp = 0, nlow = 0;
            int node = scene.root;
            const int n_int = scene.n_tri - 1;
            int budget = 2 * scene.n_tri + 64;
            while (--budget > 0) {
                if (node >= n_int || ~node >= scene.n_tri) break;
                if (node >= 0) {
                    if (COUNT) ++visits;
                    const float4* nd = scene.nodes + 4 * node;
                    float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
                    float tl, tr;
                    bool hl = cone_box(c, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tcull, tl);
                    bool hr = cone_box(c, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tcull, tr);
                    int cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
                    if (hl && hr) {
                        const bool lfirst = tl <= tr;
                        int nearc = lfirst ? cl : cr;
                        int2 farc = make_int2(lfirst ? cr : cl, __float_as_int(lfirst ? tr : tl));
                        if (sp - nlow > ring_mask) {
                            if (nlow < kMaxSpill) spill[nlow] = my[(nlow & ring_mask) * stride];
                            ++nlow;
                        }
                        my[(sp & ring_mask) * stride] = farc;
                        ++sp;
                        node = nearc;
                        continue;
                    }
                    if (hl) { node = cl; continue; }
                    if (hr) { node = cr; continue; }
                } else {
                    if (n == kCandMax) {  // too many: the subrays traverse on their own
                        n = -1;
                        break;
                    }
                    out[1 + n] = ~node;
                    ++n;
                    double tc = cover_distance(c, scene.tris, ~node);
                    if (tc < INFINITY) {
                        float tf = (float)tc;
                        if ((double)tf < tc) tf = nextafterf(tf, INFINITY);
                        tcull = fminf(tcull, tf);
                    }
                }
                // pop the next node that can still hold a closest hit
                bool found = false;
                while (sp > 0) {
                    --sp;
                    int2 e;
                    if (sp < nlow) {
                        e = sp < kMaxSpill ? spill[sp] : make_int2(-1, 0);
                        nlow = sp;
                    } else {
                        e = my[(sp & ring_mask) * stride];
                    }
                    if (__int_as_float(e.y) <= tcull) {
                        node = e.x;
                        found = true;
                        break;
                    }
                }
                if (!found) break;
            }
            if (budget <= 0) n = -1;
        }
        out[0] = n;
    }
    if (COUNT) {
        unsigned long long v = (unsigned long long)visits;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(counts + 1, v);
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

hipError_t launch_cone(const SceneDev& scene, double tan_max, const PulsesDev& pulses, int* cand, long long first,
                       long long count, const LaunchCfg& cfg, unsigned long long* counts, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const int block = 64 * cfg.block_waves;
    unsigned grid = (unsigned)((count + block - 1) / block);
    size_t lds = sizeof(int2) * (size_t)cfg.stack_lds * block;
    int mask = cfg.stack_lds - 1;
    if (counts)
        hipLaunchKernelGGL(k_cone<true>, dim3(grid), dim3(block), lds, stream, scene, tan_max, pulses, cand, first,
                           count, mask, counts);
    else
        hipLaunchKernelGGL(k_cone<false>, dim3(grid), dim3(block), lds, stream, scene, tan_max, pulses, cand, first,
                           count, mask, counts);
    return hipGetLastError();
}

}  // namespace vls
