// Adjoint of the waveform with respect to per-triangle reflectance and vertex
// heights, for a loss L(wf) whose gradient G = dL/dwf is given.
//
// Hit selection is discrete and held fixed: the subray's triangle comes from the
// forward pass, and the window origin t0 is the forward's (a fixed input).  Per
// subray the continuous state is recomputed rather than stored:
//   R   = n.(a - O) / n.d            (range to the triangle's plane; n = e1 x e2)
//   cos = |n.d| / |n|                (incidence, Sec. 5.2)
//   P   = C w rho cos / R^2          (Eq. 7 with a Lambertian extended target)
//   tau = 2 R / c                    (two-way travel time, Sec. 3.4)
//   wf_j += P p(t0 + j bin - tau)    (Sec. 3.4, Eq. 3 or a Gaussian pulse)
// so with gP = sum_j G_j p(s_j) and gD = sum_j G_j p'(s_j):
//   dL/dtau = -P gD,   dL/dR = dL/dtau 2/c - gP 2P/R,
//   dL/drho = gP C w cos / R^2,   dL/dcos = gP C w rho / R^2,
//   dR/dv_i = b_i n / (n.d) (b_i: barycentric weight of vertex i at the hit),
//   dcos/dn = sgn(n.d) (d/|n| - (n.d) n/|n|^3), with dn = dv0 x (e1 - e2),
//   dn = dv1 x e2, dn = e1 x dv2 for moves of the three vertices.
// Only the z (height) components of the vertex gradients are kept.  Lanes of a
// wavefront that share a triangle are summed in the wavefront first, so each
// (wavefront, triangle) pair issues one atomic per gradient entry.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "device_common.h"
#include "vls_internal.h"

namespace vls {
namespace {

using namespace dev;

struct Grads {
    double grho, gz[3];
};

// Gradient contributions of one subray that hit triangle `tri`.
__device__ __forceinline__ bool subray_grads(const SceneDev& scene, const ScannerDev& sc, const Ray& r, int tri,
                                             double w, double t0, const float* __restrict__ G, Grads& out)
{
#pragma clang fp contract(off)
    const int32_t* ti = scene.tri_idx + 3 * (long long)tri;
    const float* V = scene.verts;
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = V[3 * (long long)ti[0] + i];
        b[i] = V[3 * (long long)ti[1] + i];
        c[i] = V[3 * (long long)ti[2] + i];
    }
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double nd = n[0] * r.D[0] + n[1] * r.D[1] + n[2] * r.D[2];
    double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    if (nd == 0.0 || nn == 0.0) return false;
    double R = (n[0] * (a[0] - r.O[0]) + n[1] * (a[1] - r.O[1]) + n[2] * (a[2] - r.O[2])) / nd;
    if (!(R > 0.0)) return false;
    double X[3] = {r.O[0] + R * r.D[0] - a[0], r.O[1] + R * r.D[1] - a[1], r.O[2] + R * r.D[2] - a[2]};
    // barycentric weights of the hit point: X - a = u e1 + v e2
    double xe2[3] = {X[1] * e2[2] - X[2] * e2[1], X[2] * e2[0] - X[0] * e2[2], X[0] * e2[1] - X[1] * e2[0]};
    double e1x[3] = {e1[1] * X[2] - e1[2] * X[1], e1[2] * X[0] - e1[0] * X[2], e1[0] * X[1] - e1[1] * X[0]};
    double u = (xe2[0] * n[0] + xe2[1] * n[1] + xe2[2] * n[2]) / nn;
    double v = (e1x[0] * n[0] + e1x[1] * n[1] + e1x[2] * n[2]) / nn;
    double bw[3] = {1.0 - u - v, u, v};
    double len = sqrt(nn);
    double cosv = fabs(nd) / len;
    double rho = scene.refl[tri];
    double base = sc.power_c * w / (R * R);
    // surface response f and df/dcos: cos, or the Phong-type specular response
    double f = cosv, df = 1.0;
    if (scene.spec_k) {
        const double ks = scene.spec_k[tri], ns = scene.spec_n[tri];
        const double c2 = 2.0 * cosv * cosv - 1.0;
        f = (1.0 - ks) * cosv + ks * (c2 > 0.0 ? pow(c2, ns) : 0.0);
        df = (1.0 - ks) + (c2 > 0.0 && ns != 0.0 ? ks * ns * pow(c2, ns - 1.0) * 4.0 * cosv : 0.0);
    }
    double P = base * rho * f;
    double tau = round_trip_ns(R);
    double rel = tau - t0;
    // bins inside the pulse support around this echo
    double lo = ceil((rel - sc.cut_lo) / sc.bin_d), hi = floor((rel + sc.cut_hi) / sc.bin_d);
    int jl = (int)fmax(lo, 0.0), jh = (int)fmin(hi, (double)(sc.n_bins - 1));
    float rh = (float)rel, rl = (float)(rel - (double)rh);
    float gP = 0.0f, gD = 0.0f;
    const float inv_s2 = -2.0f * sc.neg_k * 0.6931471805599453f;  // 1 / sigma^2 for the Gaussian
    for (int j = jl; j <= jh; ++j) {
        double xd = (double)j * sc.bin_d;
        float xh = (float)xd, xl = (float)(xd - (double)xh);
        float s = (xh - rh) + (xl - rl);
        float p, dp;
        if (sc.shape == 0) {
            p = __builtin_amdgcn_exp2f(s * s * sc.neg_k);
            dp = -s * inv_s2 * p;
        } else {
            float x = s * sc.inv_tau;
            float e = s > 0.0f ? __builtin_amdgcn_exp2f(x * sc.neg_k) : 0.0f;
            p = x * x * e;
            dp = (2.0f * x - x * x) * e * sc.inv_tau;
        }
        float g = G[j];
        gP += g * p;
        gD += g * dp;
    }
    double gtau = -P * (double)gD;
    double gR = gtau * 2.0 / kCmPerNs - (double)gP * 2.0 * P / R;
    double gcos = (double)gP * base * rho * df;
    out.grho = (double)gP * base * f;
    // through R: dR/dv_i = b_i n / n.d (z component)
    for (int i = 0; i < 3; ++i) out.gz[i] = gR * bw[i] * n[2] / nd;
    // through cos: gradient with respect to n, then to the vertices
    double sg = nd >= 0.0 ? 1.0 : -1.0;
    double gn[3];
    for (int i = 0; i < 3; ++i) gn[i] = gcos * sg * (r.D[i] / len - nd * n[i] / (nn * len));
    double d12[3] = {e1[0] - e2[0], e1[1] - e2[1], e1[2] - e2[2]};
    out.gz[0] += d12[0] * gn[1] - d12[1] * gn[0];   // ((e1 - e2) x gn).z
    out.gz[1] += e2[0] * gn[1] - e2[1] * gn[0];     // (e2 x gn).z
    out.gz[2] += gn[0] * e1[1] - gn[1] * e1[0];     // (gn x e1).z
    return true;
}

__global__ __launch_bounds__(256) void k_fill_f32(float* p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_backward(SceneDev scene, ScannerDev sc, PulsesDev pulses,
                                                  const int32_t* __restrict__ sub_tri, int sub_stride,
                                                  const float* __restrict__ grad_wf, float* grad_refl,
                                                  float* grad_z, long long count)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int waves = blockDim.x / kWave;
    long long wave = (long long)blockIdx.x * waves + threadIdx.x / kWave;
    long long p0 = wave * sc.P_w;
    if (p0 >= count) return;
    long long left = count - p0;
    const int npw = left < sc.P_w ? (int)left : sc.P_w;
    const int S = sc.S;
    const int pl = lane / S, k = lane - pl * S;
    int tri = -1;
    Grads g;
    g.grho = g.gz[0] = g.gz[1] = g.gz[2] = 0.0;
    if (pl < npw) {
        long long p = p0 + pl;
        int t = sub_tri[p * sub_stride + k];
        double t0 = pulses.t0_in[p];
        if (t >= 0 && t < scene.n_tri && !isnan(t0)) {
            Ray r;
            const double* pat = sc.pattern + 5 * k;
            if (setup_ray(pulses.origins + 3 * p, pulses.dirs + 3 * p, pat, r) &&
                subray_grads(scene, sc, r, t, pat[4], t0, grad_wf + p * sc.n_bins, g))
                tri = t;
        }
    }
    // sum the contributions of lanes that share a triangle, one atomic per entry
    unsigned long long todo = __ballot(tri >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int t = __builtin_amdgcn_readlane(tri, leader);
        const bool mine = tri == t;
        todo &= ~__ballot(mine);
        float sr = wave_sum_f(mine ? (float)g.grho : 0.0f);
        float s0 = wave_sum_f(mine ? (float)g.gz[0] : 0.0f);
        float s1 = wave_sum_f(mine ? (float)g.gz[1] : 0.0f);
        float s2 = wave_sum_f(mine ? (float)g.gz[2] : 0.0f);
        if (lane == leader) {
            const int32_t* ti = scene.tri_idx + 3 * (long long)t;
            if (grad_refl) unsafeAtomicAdd(grad_refl + t, sr);
            if (grad_z) {
                unsafeAtomicAdd(grad_z + ti[0], s0);
                unsafeAtomicAdd(grad_z + ti[1], s1);
                unsafeAtomicAdd(grad_z + ti[2], s2);
            }
        }
    }
}

// Deterministic form: instead of atomics, every subray slot e (pulse p, subray
// k: e = p S + k) writes four entries, 4 e + c: c = 0 its reflectance
// contribution keyed by its triangle, c = 1..3 its height contributions keyed
// by the triangle's vertices (key = kind << id_bits | id, kind 0 reflectance,
// 1 height; slots without a hit or an unrequested gradient get the key
// `none`), with the contribution's FP32 bits as the entry's value.  A stable
// sort by key then puts each parameter's contributions together in entry
// order, and one thread per run sums them in that order.
__global__ __launch_bounds__(256) void k_backward_entries(SceneDev scene, ScannerDev sc, PulsesDev pulses,
                                                          const int32_t* __restrict__ sub_tri, int sub_stride,
                                                          const float* __restrict__ grad_wf, bool want_refl,
                                                          bool want_z, int id_bits, unsigned long long none,
                                                          unsigned long long* __restrict__ keys,
                                                          int32_t* __restrict__ vals, long long count)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int waves = blockDim.x / kWave;
    long long wave = (long long)blockIdx.x * waves + threadIdx.x / kWave;
    long long p0 = wave * sc.P_w;
    if (p0 >= count) return;
    long long left = count - p0;
    const int npw = left < sc.P_w ? (int)left : sc.P_w;
    const int S = sc.S;
    const int pl = lane / S, k = lane - pl * S;
    if (pl >= npw) return;
    const long long p = p0 + pl;
    int tri = -1;
    Grads g;
    g.grho = g.gz[0] = g.gz[1] = g.gz[2] = 0.0;
    int t = sub_tri[p * sub_stride + k];
    double t0 = pulses.t0_in[p];
    if (t >= 0 && t < scene.n_tri && !isnan(t0)) {
        Ray r;
        const double* pat = sc.pattern + 5 * k;
        if (setup_ray(pulses.origins + 3 * p, pulses.dirs + 3 * p, pat, r) &&
            subray_grads(scene, sc, r, t, pat[4], t0, grad_wf + p * sc.n_bins, g))
            tri = t;
    }
    const long long e = 4 * (p * S + k);
    const int32_t* ti = scene.tri_idx + 3 * (long long)(tri >= 0 ? tri : 0);
    keys[e] = tri >= 0 && want_refl ? (unsigned long long)tri : none;
    vals[e] = __float_as_int((float)g.grho);
    for (int c = 0; c < 3; ++c) {
        keys[e + 1 + c] = tri >= 0 && want_z ? (1ull << id_bits) | (unsigned long long)ti[c] : none;
        vals[e + 1 + c] = __float_as_int((float)g.gz[c]);
    }
}

// One thread per sorted entry; the first entry of each run of equal keys sums
// the run's contributions in entry order (FP64) and writes the parameter.
__global__ __launch_bounds__(256) void k_segment_sums(const unsigned long long* __restrict__ keys,
                                                      const int32_t* __restrict__ vals, long long n, int id_bits,
                                                      unsigned long long none, float* grad_refl, float* grad_z)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long key = keys[i];
    if (key == none || (i > 0 && keys[i - 1] == key)) return;
    double sum = 0.0;
    for (long long j = i; j < n && keys[j] == key; ++j) sum += (double)__int_as_float(vals[j]);
    const unsigned long long id = key & ((1ull << id_bits) - 1);
    if ((key >> id_bits) == 0) grad_refl[id] = (float)sum;
    else grad_z[id] = (float)sum;
}

}  // namespace

// Bits of a parameter index in the deterministic form's keys (ids below
// max(n_tri, n_vert)), and the sort passes (8 bits each) that cover the kind bit
// and the `none` key.
static int backward_id_bits(long long n_tri, long long n_vert)
{
    long long m = n_tri > n_vert ? n_tri : n_vert;
    int b = 1;
    while ((1ll << b) < m) ++b;
    return b;
}

size_t backward_det_bytes(long long n_pulses, int S)
{
    const long long n = 4 * n_pulses * (long long)S;
    const size_t a = (size_t)n;
    return 2 * 8 * a + 2 * 4 * a + 4 * (size_t)radix_sort_hist_words(n) + 4 * 256;
}

hipError_t launch_backward_det(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                               const int32_t* sub_tri, int sub_stride, const float* grad_wf, float* grad_refl,
                               float* grad_z, long long n_vert, const LaunchCfg& cfg, void* ws, hipStream_t stream)
{
    if (grad_refl && scene.n_tri > 0)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((scene.n_tri + 255) / 256)), dim3(256), 0, stream, grad_refl,
                           (long long)scene.n_tri);
    if (grad_z && n_vert > 0)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n_vert + 255) / 256)), dim3(256), 0, stream, grad_z, n_vert);
    if (pulses.n <= 0 || scene.n_tri <= 0) return hipGetLastError();
    const long long n = 4 * pulses.n * (long long)sc.S;
    const int id_bits = backward_id_bits(scene.n_tri, n_vert);
    const unsigned long long none = (2ull << id_bits) | ((1ull << id_bits) - 1);  // kind 2: after every real key
    const int passes = (id_bits + 2 + 7) / 8;
    unsigned char* w = static_cast<unsigned char*>(ws);
    auto* keys = reinterpret_cast<unsigned long long*>(w);
    auto* keys2 = keys + n;
    auto* vals = reinterpret_cast<int32_t*>(keys2 + n);
    int32_t* vals2 = vals + n;
    unsigned* hist = reinterpret_cast<unsigned*>(vals2 + n);
    const int block = cfg.block_waves * kWave;
    long long waves = (pulses.n + sc.P_w - 1) / sc.P_w;
    unsigned grid = (unsigned)((waves + cfg.block_waves - 1) / cfg.block_waves);
    // every entry is written: each slot (p < n_pulses, k < S) is one lane of one wavefront
    hipLaunchKernelGGL(k_backward_entries, dim3(grid), dim3(block), 0, stream, scene, sc, pulses, sub_tri, sub_stride,
                       grad_wf, grad_refl != nullptr, grad_z != nullptr, id_bits, none, keys, vals, pulses.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = radix_sort_pairs(keys, vals, keys2, vals2, hist, n, passes, stream)) != hipSuccess) return e;
    // the sort alternates between the two pairs of arrays: an odd number of
    // passes leaves the result in the second
    const unsigned long long* ks = passes & 1 ? keys2 : keys;
    const int32_t* vs = passes & 1 ? vals2 : vals;
    hipLaunchKernelGGL(k_segment_sums, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ks, vs, n, id_bits,
                       none, grad_refl, grad_z);
    return hipGetLastError();
}

hipError_t launch_backward(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                           const int32_t* sub_tri, int sub_stride, const float* grad_wf, float* grad_refl,
                           float* grad_z, long long n_vert, const LaunchCfg& cfg, hipStream_t stream)
{
    if (grad_refl && scene.n_tri > 0)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((scene.n_tri + 255) / 256)), dim3(256), 0, stream, grad_refl,
                           (long long)scene.n_tri);
    if (grad_z && n_vert > 0)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n_vert + 255) / 256)), dim3(256), 0, stream, grad_z, n_vert);
    if (pulses.n > 0 && scene.n_tri > 0) {
        const int block = cfg.block_waves * kWave;
        long long waves = (pulses.n + sc.P_w - 1) / sc.P_w;
        unsigned grid = (unsigned)((waves + cfg.block_waves - 1) / cfg.block_waves);
        hipLaunchKernelGGL(k_backward, dim3(grid), dim3(block), 0, stream, scene, sc, pulses, sub_tri, sub_stride,
                           grad_wf, grad_refl, grad_z, pulses.n);
    }
    return hipGetLastError();
}

}  // namespace vls
