// Scene parts placed by affine maps (Sec. 3.5: one part loaded several times
// and moved by transforms; Sec. 5.1: primitives rotate, scale and translate).
//
// Each instance of a part contributes the part's triangles in the scene's
// frame: vertices x -> A x + t, evaluated in FP64 as ((A_i0 x + A_i1 y) +
// A_i2 z) + t_i with contraction off and rounded once to FP32; vertex indices
// offset by the instance's first vertex; the part's reflectance.  Instances
// are laid out in their order, so instance j's triangles are the ids
// [tri_off_j, tri_off_j + part triangles).  The scene built from the result is
// an ordinary one: the hot path is unchanged.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "vls_internal.h"

namespace vls {
namespace {

// Vertices of the k instances of one part: thread q = instance slot * nv + vertex.
// aff: [k][12] rows (A_i0, A_i1, A_i2, t_i); voff: [k] first scene vertex.
__global__ __launch_bounds__(256) void k_instance_verts(const float* __restrict__ v, long long nv,
                                                        const double* __restrict__ aff,
                                                        const long long* __restrict__ voff, long long k,
                                                        float* __restrict__ out)
{
#pragma clang fp contract(off)
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= k * nv) return;
    const long long j = q / nv, i = q - j * nv;
    const double x = v[3 * i], y = v[3 * i + 1], z = v[3 * i + 2];
    const double* a = aff + 12 * j;
    float* o = out + 3 * (voff[j] + i);
    for (int r = 0; r < 3; ++r) {
        double w = a[4 * r] * x;
        w = w + a[4 * r + 1] * y;
        w = w + a[4 * r + 2] * z;
        w = w + a[4 * r + 3];
        o[r] = (float)w;
    }
}

// Triangles of the k instances of one part: indices offset by the instance's
// first vertex, reflectance copied.  An index outside [0, nv) sets *bad.
__global__ __launch_bounds__(256) void k_instance_tris(const int32_t* __restrict__ t, const float* __restrict__ refl,
                                                       long long nt, long long nv,
                                                       const long long* __restrict__ voff,
                                                       const long long* __restrict__ toff, long long k,
                                                       int32_t* __restrict__ out_t, float* __restrict__ out_r,
                                                       unsigned* __restrict__ bad)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= k * nt) return;
    const long long j = q / nt, i = q - j * nt;
    const long long dst = toff[j] + i;
    bool ok = true;
    for (int c = 0; c < 3; ++c) {
        const int32_t id = t[3 * i + c];
        ok = ok && id >= 0 && (long long)id < nv;
        out_t[3 * dst + c] = ok ? (int32_t)(voff[j] + id) : 0;
    }
    out_r[dst] = refl[i];
    if (!ok) atomicOr(bad, 1u);
}

}  // namespace

hipError_t launch_instances(const float* v, const int32_t* t, const float* refl, long long nv, long long nt,
                            const double* aff, const long long* voff, const long long* toff, long long k,
                            float* out_v, int32_t* out_t, float* out_r, unsigned* bad, hipStream_t stream)
{
    if (k <= 0) return hipSuccess;
    if (nv > 0)
        hipLaunchKernelGGL(k_instance_verts, dim3((unsigned)((k * nv + 255) / 256)), dim3(256), 0, stream, v, nv, aff,
                           voff, k, out_v);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nt > 0)
        hipLaunchKernelGGL(k_instance_tris, dim3((unsigned)((k * nt + 255) / 256)), dim3(256), 0, stream, t, refl, nt,
                           nv, voff, toff, k, out_t, out_r, bad);
    return hipGetLastError();
}

}  // namespace vls
