// Device helpers shared by the library's kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "vls_internal.h"

namespace vls {
namespace dev {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Whole-wavefront reductions with DPP (data-parallel primitives): pairs and
// quads, half-rows and rows by mirroring, then row broadcasts of lanes 15 and
// 31; lane 63 ends with the result, which readlane makes wave-uniform.  Every
// lane must be active.  Each step is one DPP move plus the operation.
#define VLS_DPP_STEPS(STEP) STEP(0xB1, 0xF) STEP(0x4E, 0xF) STEP(0x141, 0xF) STEP(0x140, 0xF) STEP(0x142, 0xA) STEP(0x143, 0xC)

__device__ __forceinline__ int wave_bcast63_i(int v) { return __builtin_amdgcn_readlane(v, 63); }

__device__ __forceinline__ float wave_min_f(float v)
{
    const int id = __float_as_int(INFINITY);
#define VLS_STEP(C, M) v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(id, __float_as_int(v), C, M, 0xF, false)));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return __int_as_float(wave_bcast63_i(__float_as_int(v)));
}

__device__ __forceinline__ float wave_max_f(float v)
{
    const int id = __float_as_int(-INFINITY);
#define VLS_STEP(C, M) v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(id, __float_as_int(v), C, M, 0xF, false)));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return __int_as_float(wave_bcast63_i(__float_as_int(v)));
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#define VLS_STEP(C, M) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, M, 0xF, false));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return __int_as_float(wave_bcast63_i(__float_as_int(v)));
}

__device__ __forceinline__ int wave_min_i(int v)
{
#define VLS_STEP(C, M) v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, C, M, 0xF, false));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return wave_bcast63_i(v);
}

__device__ __forceinline__ int wave_max_i(int v)
{
#define VLS_STEP(C, M) v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, C, M, 0xF, false));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return wave_bcast63_i(v);
}

__device__ __forceinline__ double wave_min_d(double v)
{
    const int id_lo = __double2loint(INFINITY), id_hi = __double2hiint(INFINITY);
#define VLS_STEP(C, M)                                                                         \
    v = fmin(v, __hiloint2double(__builtin_amdgcn_update_dpp(id_hi, __double2hiint(v), C, M, 0xF, false), \
                                 __builtin_amdgcn_update_dpp(id_lo, __double2loint(v), C, M, 0xF, false)));
    VLS_DPP_STEPS(VLS_STEP)
#undef VLS_STEP
    return __hiloint2double(wave_bcast63_i(__double2hiint(v)), wave_bcast63_i(__double2loint(v)));
}

// Half-wavefront reductions: the same steps without the last broadcast, so lane
// 31 ends with the result over lanes 0-31 and lane 63 with that over lanes
// 32-63; each lane gets its own half's result.
#define VLS_DPP_HALF_STEPS(STEP) STEP(0xB1, 0xF) STEP(0x4E, 0xF) STEP(0x141, 0xF) STEP(0x140, 0xF) STEP(0x142, 0xA)

__device__ __forceinline__ int half_pick_i(int v)
{
    const int a = __builtin_amdgcn_readlane(v, 31), b = __builtin_amdgcn_readlane(v, 63);
    return (threadIdx.x & 32) ? b : a;
}

__device__ __forceinline__ float half_max_f(float v)
{
    const int id = __float_as_int(-INFINITY);
#define VLS_STEP(C, M) v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(id, __float_as_int(v), C, M, 0xF, false)));
    VLS_DPP_HALF_STEPS(VLS_STEP)
#undef VLS_STEP
    return __int_as_float(half_pick_i(__float_as_int(v)));
}

__device__ __forceinline__ double half_min_d(double v)
{
    const int id_lo = __double2loint(INFINITY), id_hi = __double2hiint(INFINITY);
#define VLS_STEP(C, M)                                                                         \
    v = fmin(v, __hiloint2double(__builtin_amdgcn_update_dpp(id_hi, __double2hiint(v), C, M, 0xF, false), \
                                 __builtin_amdgcn_update_dpp(id_lo, __double2loint(v), C, M, 0xF, false)));
    VLS_DPP_HALF_STEPS(VLS_STEP)
#undef VLS_STEP
    return __hiloint2double(half_pick_i(__double2hiint(v)), half_pick_i(__double2loint(v)));
}

// Value of lane l - 1 (lane 0 gets `edge`) and of lane l + 1 (lane 63 gets `edge`).
__device__ __forceinline__ float lane_prev_f(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_next_f(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_read_f(float v, int lane) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane)); }

__device__ __forceinline__ unsigned lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

struct Ray {
    double O[3];
    double D[3];
    double Sx, Sy, Sz;  // shear of the watertight test: the ray runs along +kz
    int kz;
    float d32[3];       // direction rounded to FP32 (shading)
};

// FP32 slab constants of the box test, padded outward against the rounding of
// the FP32 ray.
struct RayBox {
    float inv[3];
    float oim[3];  // (O + pad) * inv : lower planes moved outward
    float oip[3];  // (O - pad) * inv : upper planes moved outward
};

// Duff et al. 2017 orthonormal basis; FP64 subray direction and shear.
// FP contraction is off wherever FP64 results decide a hit, so every product
// and sum is rounded exactly as written.
//
// The pulse's part: the unit axis n and the two scalars a, b from which the
// basis vectors u, v follow (with s = sign of n_z):
//   u = (1 + s n_x^2 a, s b, -s n_x),  v = (b, s + n_y^2 a, -n_y).
// False for a zero or non-finite direction.  The cone pass computes it once
// per pulse and hands it to the fused kernel in this layout.
struct Basis {
    double n[3];
    double a, b;
};

__device__ __forceinline__ bool pulse_basis(const float* __restrict__ d32, Basis& B)
{
#pragma clang fp contract(off)
    double dx = d32[0], dy = d32[1], dz = d32[2];
    double len = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(len > 0.0) || !(len < INFINITY)) return false;
    B.n[0] = dx / len;
    B.n[1] = dy / len;
    B.n[2] = dz / len;
    double sgn = copysign(1.0, B.n[2]);
    B.a = -1.0 / (sgn + B.n[2]);
    B.b = B.n[0] * B.n[1] * B.a;
    return true;
}

// The subray's part: direction from the pattern entry (cos a, sin a, cos phi,
// sin phi), dominant axis and shear.  False for a non-finite origin.
__device__ __forceinline__ bool setup_ray_b(const double* __restrict__ o, const Basis& B,
                                            const double* __restrict__ pat, Ray& r)
{
#pragma clang fp contract(off)
    const double* n = B.n;
    const double a = B.a, b = B.b;
    double sgn = copysign(1.0, n[2]);
    double u[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    double v[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    double ca = pat[0], sa = pat[1], cp = pat[2], sp = pat[3];
    double omax = 0.0;
    for (int i = 0; i < 3; ++i) {
        r.D[i] = ca * n[i] + sa * (cp * u[i] + sp * v[i]);
        r.O[i] = o[i];
        r.d32[i] = (float)r.D[i];
        omax = fmax(omax, fabs(o[i]));
    }
    if (!(omax < INFINITY)) return false;
    int kz = 0;
    double dmax = fabs(r.D[0]);
    if (fabs(r.D[1]) > dmax) {
        kz = 1;
        dmax = fabs(r.D[1]);
    }
    if (fabs(r.D[2]) > dmax) kz = 2;
    // kx, ky follow kz cyclically.  The winding-preserving swap of kx and ky for a
    // negative D[kz] is left out: the test is two-sided, and the swap would only
    // negate U, V, W, det and T exactly, leaving every decision and t unchanged.
    // Components are picked by selects, not by a run-time array index (which
    // would place the array in scratch memory).
    const double az = kz == 0 ? r.D[0] : (kz == 1 ? r.D[1] : r.D[2]);
    const double ax = kz == 0 ? r.D[1] : (kz == 1 ? r.D[2] : r.D[0]);
    const double ay = kz == 0 ? r.D[2] : (kz == 1 ? r.D[0] : r.D[1]);
    r.kz = kz;
    r.Sx = ax / az;
    r.Sy = ay / az;
    r.Sz = 1.0 / az;
    return true;
}

__device__ __forceinline__ bool setup_ray(const double* __restrict__ o, const float* __restrict__ d32,
                                          const double* __restrict__ pat, Ray& r)
{
    Basis B;
    return pulse_basis(d32, B) && setup_ray_b(o, B, pat, r);
}

// A basis stored by the cone pass ([5] doubles: n, a, b; n_x NaN for a pulse
// whose direction is zero or non-finite).
__device__ __forceinline__ bool load_basis(const double* __restrict__ stored, Basis& B)
{
    B.n[0] = stored[0];
    B.n[1] = stored[1];
    B.n[2] = stored[2];
    B.a = stored[3];
    B.b = stored[4];
    return !isnan(B.n[0]);
}

// pad covers the FP32 rounding of origin, direction and slab arithmetic
__device__ __forceinline__ void setup_box(const Ray& r, float scene_mag, RayBox& b)
{
    double omax = fmax(fmax(fabs(r.O[0]), fabs(r.O[1])), fabs(r.O[2]));
    double pad = (omax + (double)scene_mag + 1.0) * 1.9073486328125e-06;  // 2^-19
    for (int i = 0; i < 3; ++i) {
        float di = r.d32[i];
        if (fabsf(di) < 1e-30f) di = copysignf(1e-30f, di);
        float inv = 1.0f / di;
        b.inv[i] = inv;
        b.oim[i] = (float)(r.O[i] + pad) * inv;
        b.oip[i] = (float)(r.O[i] - pad) * inv;
    }
}

// Output number c of the SplitMix64 sequence seeded with `seed` (Steele, Lea &
// Flood 2014): the state after c + 1 steps of the Weyl increment, mixed.  Any
// output is reached directly, so parallel draws need no shared state.
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A uniform number in (0, 1]: ((x >> 11) + 1) 2^-53 of output c.
__device__ __forceinline__ double sm_uniform(uint64_t seed, uint64_t c)
{
    return (double)((sm64(seed, c) >> 11) + 1) * (1.0 / 9007199254740992.0);
}

// Round-trip time in ns of a range R in m, 2 R / c (Sec. 3.4), as a product with
// the double nearest to 2 / c (a division would cost an FP64 divide sequence).
constexpr double kNsPerRoundTripM = 2.0 / kCmPerNs;
__device__ __forceinline__ double round_trip_ns(double R) { return R * kNsPerRoundTripM; }

// Outgoing pulse at offset s (ns): unit-peak Gaussian (SHAPE 0), or Eq. 3
// (s/tau)^2 exp(-s/tau) (SHAPE 1).  exp2 is the hardware instruction: results
// below 2^-126 flush to zero, far under any bin that matters.
template <int SHAPE>
__device__ __forceinline__ float pulse_shape(const ScannerDev& sc, float s)
{
    if (SHAPE == 0) return __builtin_amdgcn_exp2f(s * s * sc.neg_k);
    float x = s * sc.inv_tau;
    return s > 0.0f ? x * x * __builtin_amdgcn_exp2f(x * sc.neg_k) : 0.0f;
}

}  // namespace dev
}  // namespace vls
