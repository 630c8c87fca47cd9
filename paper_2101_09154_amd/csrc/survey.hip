// Pulses generated on the GPU from a survey (Sec. 3.2 platforms, Sec. 3.3 scan
// deflectors), so that a scan needs no host arrays of origins and directions.
//
// The paper describes the platforms and deflectors and their patterns but gives
// no formulas; the model here: pulse k leaves at t = t0 + k / prf; a Multicopter
// with smooth turns flies coordinated turns on arcs tangent to its legs (radius
// v^2 / (g tan b)), banked toward each turn's centre, at its cruise speed
// between the ramps from and to rest at the ends of the path; a LinearPath
// platform covers its polyline of waypoints at constant speed from t = 0, stays
// level, faces the current leg's horizontal direction, and stays at the last
// waypoint afterwards (one waypoint: static, facing +x).  In the platform frame
// (x forward, y left, z up) the beam points, for an across-track angle a, along
// (0, sin a, -cos a), with a = -A + 2A frac(f t) (polygon mirror: parallel lines
// of even density), A sin(2 pi f t) (swinging mirror: a zig-zag, denser at the
// extremes) or -A + 2A (k mod N) / (N - 1) (fibre array: N fixed directions
// fired in turn); a Palmer (conic) scanner points along (sin A cos p,
// sin A sin p, -cos A), p = 2 pi frac(f t).  Platform noise adds independent
// N(0, sigma^2) offsets per axis to the origin: Box-Muller on uniforms
// ((x >> 11) + 1) 2^-53 of SplitMix64 (Steele, Lea & Flood 2014) outputs
// number 6k + 2 axis and 6k + 2 axis + 1 of the sequence seeded with the
// survey's seed, so any pulse can be generated on its own.
//
// One thread per pulse; all arithmetic in FP64, directions stored as FP32.  The
// per-leg table (waypoint, cumulative length, cos and sin of the heading) is
// computed on the host.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "device_common.h"

namespace vls {
namespace {

using dev::sm_uniform;

// tab: per waypoint i, [x, y, z, cumulative length, cos yaw, sin yaw] of the
// leg that starts there (the last entry's yaw is unused).
// Multicopter leg (Sec. 3.2: speeds up and slows down, stops at each
// waypoint): distance covered tau in [0, T] seconds into a leg of length L and
// duration T, from rest to rest at acceleration a and cruise speed v.
__device__ __forceinline__ double copter_distance(double L, double T, double v, double a, double tau)
{
#pragma clang fp contract(off)
    if (tau <= 0.0) return 0.0;
    if (tau >= T) return L;
    const double vmax = v * v / a <= L ? v : sqrt(a * L);  // speed at the end of the ramp
    const double ramp = vmax / a;
    if (tau <= ramp) return 0.5 * a * tau * tau;
    const double rest = T - tau;
    if (rest <= ramp) return L - 0.5 * a * rest * rest;
    return 0.5 * a * ramp * ramp + vmax * (tau - ramp);
}

__global__ __launch_bounds__(256) void k_generate(SurveyDev sv, const double* __restrict__ tab, long long first,
                                                  long long count, double* __restrict__ origins,
                                                  float* __restrict__ dirs)
{
#pragma clang fp contract(off)
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const long long k = first + q;
    const double t = sv.t0 + (double)k / sv.prf;
    double pos[3] = {tab[0], tab[1], tab[2]};
    double cy = 1.0, sy = 0.0, lean = 0.0;
    if (sv.n_wp >= 2 && sv.platform == 2) {
        // smooth turns: path length covered (ramp up, cruise, ramp down), then
        // the piece that holds it (the last piece starting at or before it)
        const double v = sv.speed, acc = sv.accel, tr = v / acc;
        double sg;
        if (t <= 0.0) sg = 0.0;
        else if (t <= tr) sg = 0.5 * acc * t * t;
        else if (t < sv.t_end - tr) sg = 0.5 * acc * tr * tr + v * (t - tr);
        else if (t < sv.t_end) sg = sv.path_len - 0.5 * acc * (sv.t_end - t) * (sv.t_end - t);
        else sg = sv.path_len;
        int lo = 0, hi = sv.n_piece - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[kSmoothRow * mid] < sg) lo = mid;
            else hi = mid - 1;
        }
        const double* pc = tab + kSmoothRow * lo;
        double l = sg - pc[0];
        if (l > pc[1]) l = pc[1];
        if (l < 0.0) l = 0.0;
        double dir[3];
        if (pc[2] == 0.0) {
            for (int i = 0; i < 3; ++i) {
                pos[i] = pc[5 + i] + l * pc[8 + i];
                dir[i] = pc[8 + i];
            }
        } else {
            // on the arc: angle l / r from its start, centre pc[5..7], tangent
            // at the start pc[8..10], toward the centre pc[11..13]
            const double ph = l / pc[3], c = cos(ph), s = sin(ph);
            for (int i = 0; i < 3; ++i) {
                pos[i] = pc[5 + i] - pc[3] * c * pc[11 + i] + pc[3] * s * pc[8 + i];
                dir[i] = c * pc[8 + i] + s * pc[11 + i];
            }
            lean = pc[4];
        }
        const double yaw = atan2(dir[1], dir[0]);
        cy = cos(yaw);
        sy = sin(yaw);
    } else if (sv.n_wp >= 2 && sv.platform == 1) {
        // the last leg starting at or before t (the first leg before it)
        int lo = 0, hi = sv.n_wp - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[8 * mid + 3] <= t) lo = mid;
            else hi = mid - 1;
        }
        const double* a = tab + 8 * lo;
        const double* b = tab + 8 * (lo + 1);
        const double T = a[4], L = a[5];
        double tau = t - a[3];
        if (tau < 0.0) tau = 0.0;
        if (tau > T) tau = T;
        const double f = copter_distance(L, T, sv.speed, sv.accel, tau) / L;
        for (int i = 0; i < 3; ++i) pos[i] = a[i] + f * (b[i] - a[i]);
        const double yaw = a[6] + (tau / T) * (a[7] - a[6]);
        cy = cos(yaw);
        sy = sin(yaw);
    } else if (sv.n_wp >= 2) {
        const double sd = sv.speed * t;
        // the last leg whose start lies at or before sd (the first leg before it)
        int lo = 0, hi = sv.n_wp - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[6 * mid + 3] <= sd) lo = mid;
            else hi = mid - 1;
        }
        const double* a = tab + 6 * lo;
        const double* b = tab + 6 * (lo + 1);
        const double len = b[3] - a[3];
        double f = len > 0.0 ? (sd - a[3]) / len : 0.0;
        if (f < 0.0) f = 0.0;
        if (f > 1.0) f = 1.0;
        for (int i = 0; i < 3; ++i) pos[i] = a[i] + f * (b[i] - a[i]);
        cy = a[4];
        sy = a[5];
    }
    if (sv.noise > 0.0) {
        for (int ax = 0; ax < 3; ++ax) {
            const uint64_t c = 6 * (uint64_t)k + 2 * (uint64_t)ax;
            const double u1 = sm_uniform(sv.seed, c), u2 = sm_uniform(sv.seed, c + 1);
            pos[ax] += sv.noise * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
        }
    }
    const double A = sv.angle;
    double ph = sv.freq * t;
    ph -= floor(ph);
    double d0, d1, d2;
    if (sv.deflector == 2) {
        const double p = 2.0 * M_PI * ph;
        d0 = sin(A) * cos(p);
        d1 = sin(A) * sin(p);
        d2 = -cos(A);
    } else {
        double ang;
        if (sv.deflector == 0) ang = -A + 2.0 * A * ph;
        else if (sv.deflector == 1) ang = A * sin(2.0 * M_PI * sv.freq * t);
        else ang = -A + 2.0 * A * (double)(k % sv.n_fibres) / (double)(sv.n_fibres - 1);
        d0 = 0.0;
        d1 = sin(ang);
        d2 = -cos(ang);
    }
    if (lean != 0.0) {
        // banked toward the turn's centre
        const double cl = cos(lean), sl = sin(lean);
        const double y = d1 * cl + d2 * sl, z = -d1 * sl + d2 * cl;
        d1 = y;
        d2 = z;
    }
    double* o = origins + 3 * q;
    float* w = dirs + 3 * q;
    o[0] = pos[0];
    o[1] = pos[1];
    o[2] = pos[2];
    w[0] = (float)(cy * d0 - sy * d1);
    w[1] = (float)(sy * d0 + cy * d1);
    w[2] = (float)d2;
}

// Ranging error (Sec. 3.7: each distance measurement carries a normally
// distributed error; mean 0 and the scanner's standard deviation here), added
// to the kept returns of pulses [first, first + count) after they are found:
// Box-Muller on the uniforms of SplitMix64 outputs 2 (p K + slot) and
// 2 (p K + slot) + 1 of the scanner's noise seed, so each return's draw is
// fixed by its pulse and slot alone.  One thread per return slot.
__global__ __launch_bounds__(256) void k_range_noise(double sigma, uint64_t seed, int K, const int32_t* __restrict__ n_ret,
                                                     float* __restrict__ ret_range, long long first, long long count)
{
#pragma clang fp contract(off)
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count * K) return;
    const long long p = first + q / K;
    const int slot = (int)(q - (q / K) * K);
    if (slot >= n_ret[p]) return;
    const uint64_t c = 2 * ((uint64_t)p * (uint64_t)K + (uint64_t)slot);
    const double u1 = sm_uniform(seed, c), u2 = sm_uniform(seed, c + 1);
    float* r = ret_range + p * K + slot;
    *r = (float)((double)*r + sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
}

}  // namespace

hipError_t launch_range_noise(const ScannerDev& sc, const int32_t* n_ret, float* ret_range, long long first,
                              long long count, hipStream_t stream)
{
    if (count <= 0 || !(sc.range_noise > 0.0)) return hipSuccess;
    const long long n = count * sc.K;
    hipLaunchKernelGGL(k_range_noise, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sc.range_noise,
                       (uint64_t)sc.noise_seed, sc.K, n_ret, ret_range, first, count);
    return hipGetLastError();
}

hipError_t launch_generate(const SurveyDev& sv, const double* tab, long long first, long long count,
                           double* origins, float* dirs, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_generate, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, sv, tab, first,
                       count, origins, dirs);
    return hipGetLastError();
}

}  // namespace vls
