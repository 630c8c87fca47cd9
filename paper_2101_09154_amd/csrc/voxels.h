// Transmissive voxels on the device (Sec. 3.5.4, Sec. 5.2): the first voxel of
// a grid that stops a subray before a given distance.
//
// Model:
//   extinction  sigma = PAD * g(|v_z|): the leaf-angle table (Table 2) gives the
//               hit probability against the beam's vertical component (its
//               horizontal one is sqrt(1 - v_z^2)); g is linear between rows
//               and held beyond the first and last;
//   depth       s = -ln(u) / sigma (Eq. 6) with u uniform in (0, 1]: one draw
//               per voxel a subray crosses, SplitMix64 output number
//               (pulse * 64 + subray) * n_voxels + voxel of the grid's seed, so
//               every draw is fixed by the subray and the voxel alone;
//   stop        the subray stops in a voxel when s is at most the length it
//               travels inside it (Sec. 5.2), at s past its entry; sigma = 0
//               lets it through;
//   walk        voxels are visited in order along the subray (Amanatides & Woo
//               1987) from where it enters the grid to where it leaves it or
//               reaches the limit (the closest triangle): consecutive
//               intersections along one ray (Sec. 5.1), without an epsilon step.
// All arithmetic in FP64 with contraction off, so every boundary decision is
// rounded as written.  The stop test s <= L equals u >= exp(-sigma L); an FP32
// estimate of that exponential settles, without the FP64 log and divide, the
// voxels whose draw lies clearly below it (no stop); every other voxel, every
// stop among them, takes the FP64 test as written.
#pragma once

#include "device_common.h"

namespace vls {
namespace dev {

// g of the leaf-angle table at |vz|.
__device__ __forceinline__ double vox_lut(const VoxDev& v, double vz)
{
#pragma clang fp contract(off)
    const double a = fabs(vz);
    const double* t = v.lut;
    const int n = v.n_lut;
    if (a <= t[0]) return t[1];
    if (a >= t[2 * (n - 1)]) return t[2 * (n - 1) + 1];
    // the last row at or below a (rows strictly increasing; row n - 1 is above a)
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[2 * mid] <= a) lo = mid;
        else hi = mid - 1;
    }
    const double x0 = t[2 * lo], x1 = t[2 * lo + 2], g0 = t[2 * lo + 1], g1 = t[2 * lo + 3];
    const double f = (a - x0) / (x1 - x0);
    return g0 + f * (g1 - g0);
}

// One axis of the walk: the current cell, the distance at which the ray leaves
// it, the distance between boundaries, the step.
struct VoxAxis {
    int i, step;
    double tmax, tdel;
};

// Entry t_in into the slab of one axis; false when the ray runs parallel to it
// outside.
__device__ __forceinline__ bool vox_clip(double o, double d, double lo, double hi, double& t_in, double& t_out)
{
#pragma clang fp contract(off)
    if (d == 0.0) return !(o < lo || o > hi);
    double t1 = (lo - o) / d, t2 = (hi - o) / d;
    if (t1 > t2) {
        const double x = t1;
        t1 = t2;
        t2 = x;
    }
    if (t1 > t_in) t_in = t1;
    if (t2 < t_out) t_out = t2;
    return true;
}

// The cell entered at distance t_in: a point on a boundary belongs to the cell
// the ray moves into.
__device__ __forceinline__ VoxAxis vox_axis(double o, double d, double t_in, double g0, double size, int n)
{
#pragma clang fp contract(off)
    VoxAxis a;
    const double q = (o + t_in * d - g0) / size;
    const double f = d < 0.0 ? ceil(q) - 1.0 : floor(q);
    a.i = f < 0.0 ? 0 : (f > (double)(n - 1) ? n - 1 : (int)f);
    if (d > 0.0) {
        a.step = 1;
        a.tmax = (g0 + size * (double)(a.i + 1) - o) / d;
        a.tdel = size / d;
    } else if (d < 0.0) {
        a.step = -1;
        a.tmax = (g0 + size * (double)a.i - o) / d;
        a.tdel = -size / d;
    } else {
        a.step = 0;
        a.tmax = INFINITY;
        a.tdel = INFINITY;
    }
    return a;
}

// The voxel (index, or -1) that stops the ray O + t D (D unit, both finite)
// before t_limit, its stop distance and sigma.  `c0` = (pulse * 64 + subray) *
// n_vox addresses the draws.  Each step leaves the current cell along one axis
// in a fixed direction, so the walk ends within nx + ny + nz steps; the loop
// bound states that.
__device__ __forceinline__ long long voxel_stop(const VoxDev& v, const double* O, const double* D, double t_limit,
                                                uint64_t c0, double& t_hit, double& sigma)
{
#pragma clang fp contract(off)
    double t_in = 0.0, t_out = t_limit;
    const double s = v.size;
    if (!vox_clip(O[0], D[0], v.origin[0], v.origin[0] + s * (double)v.nx, t_in, t_out) ||
        !vox_clip(O[1], D[1], v.origin[1], v.origin[1] + s * (double)v.ny, t_in, t_out) ||
        !vox_clip(O[2], D[2], v.origin[2], v.origin[2] + s * (double)v.nz, t_in, t_out) || !(t_in < t_out))
        return -1;
    VoxAxis X = vox_axis(O[0], D[0], t_in, v.origin[0], s, v.nx);
    VoxAxis Y = vox_axis(O[1], D[1], t_in, v.origin[1], s, v.ny);
    VoxAxis Z = vox_axis(O[2], D[2], t_in, v.origin[2], s, v.nz);
    const double g = vox_lut(v, D[2]);
    const long long plane = (long long)v.nx * v.ny;
    // the cell's index, moved by one cell along the axis of each step
    long long vi = (long long)X.i + (long long)v.nx * Y.i + plane * Z.i;
    const long long dx = X.step, dy = (long long)Y.step * v.nx, dz = (long long)Z.step * plane;
    double t = t_in;
    const int max_steps = v.nx + v.ny + v.nz + 1;
    for (int it = 0; it < max_steps && t < t_out; ++it) {
        // the axis whose boundary comes first (the lower axis on a tie)
        const int ax = Y.tmax < X.tmax ? (Z.tmax < Y.tmax ? 2 : 1) : (Z.tmax < X.tmax ? 2 : 0);
        const double tb = ax == 0 ? X.tmax : (ax == 1 ? Y.tmax : Z.tmax);
        double t_exit = tb < t_out ? tb : t_out;
        if (t_exit < t) t_exit = t;
        const float pd = v.pad[vi];
        const double sg = pd > 0.0f ? (double)pd * g : 0.0;
        if (sg > 0.0) {
            const double u = sm_uniform(v.seed, c0 + (uint64_t)vi);
            // y = 2^(-x log2 e) for x = sigma L <= 64: rounding the exponent to
            // FP32 (at most 92.4 in magnitude, so y stays normal) and the 1-ulp
            // v_exp_f32 keep y within a factor 1 +- 2^-17 of exp(-x); then
            // u < y (1 - 2^-12) gives -ln u > x + 2^-13, and the FP64 s (log and
            // divide within 2^-50 relative) exceeds L for any x below 2^36.
            const double x = sg * (t_exit - t);
            const bool below = x <= 64.0 &&
                               u < (double)__builtin_amdgcn_exp2f((float)(x * -1.4426950408889634)) *
                                       (1.0 - 0x1p-12);
            if (!below) {
                const double sd = -log(u) / sg;
                if (sd <= t_exit - t) {
                    t_hit = t + sd;
                    sigma = sg;
                    return vi;
                }
            }
        }
        t = t_exit;
        if (ax == 0) {
            X.i += X.step;
            if (X.i < 0 || X.i >= v.nx) break;
            X.tmax += X.tdel;
            vi += dx;
        } else if (ax == 1) {
            Y.i += Y.step;
            if (Y.i < 0 || Y.i >= v.ny) break;
            Y.tmax += Y.tdel;
            vi += dy;
        } else {
            Z.i += Z.step;
            if (Z.i < 0 || Z.i >= v.nz) break;
            Z.tmax += Z.tdel;
            vi += dz;
        }
    }
    return -1;
}

}  // namespace dev
}  // namespace vls
