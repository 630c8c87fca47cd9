// Echo width for gfx950 (Sec. 3.4: optionally a Gaussian is fitted to the
// waveform around each return by non-linear least squares, and its standard
// deviation is the return's width; the return's position stays the local
// maximum.  Sec. 3.6 notes the fit's cost).
//
// The samples are the return's lobe: from the return bin j outward while the
// waveform keeps falling strictly and stays at or above 2^-10 of wf[j] (a
// power-of-two scale, so FP32 and FP64 decide it alike), at most kEwHalf bins to
// each side.  The model
// A exp(-(x - mu)^2 / (2 s^2)), x = bin - j, starts from the Gaussian through
// bins j-1, j, j+1 (a parabola through their logarithms) when those lie in the
// lobe, are positive and curve downward, else from A = wf[j], mu = 0 and the
// pulse's own standard deviation; Levenberg-Marquardt with Marquardt's scaling
// then runs exactly kEwIters iterations (damping 1e-3 at the start, / 10 on an
// accepted step, * 10 on a rejected one; a trial centre farther from j than the
// lobe is long, or a width beyond twice the lobe's bins, counts as rejected).  Width = |s| bin in ns; NaN for a lobe
// of fewer than three bins or a fit that ends with A <= 0 or a non-finite s.
//
// Two launches: k_ew_list lists every kept (pulse, return) pair (one atomic per
// block of 1024 pulses) and writes NaN to every slot; k_ew_fit gives each lane one listed
// return, so every lane of a wavefront has a fit to do.  A lane caches the
// 2 kEwHalf + 1 bins around its return in LDS, bin-major ([bin][lane]), so the
// lanes of a wavefront read consecutive words, and runs the fit in FP32; each
// iteration is one pass over the lobe that yields the trial point's residual
// sum and its normal equations together.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "device_common.h"
#include "vls_internal.h"

namespace vls {
namespace {

constexpr int kEwHalf = 31;
constexpr int kEwSpan = 2 * kEwHalf + 1;
constexpr int kEwIters = 12;

constexpr int kEwListThreads = 1024;

// Lists the kept returns of pulses [first, first + count): entry = p * K + k.
// list_ctr[0] counts them (reset by the launcher); each block takes its slots
// with one atomic.  Every width slot of these pulses is set to NaN (coalesced);
// the fit overwrites the listed ones.
__global__ __launch_bounds__(kEwListThreads) void k_ew_list(const int32_t* __restrict__ n_ret, int K,
                                                            long long first, long long count,
                                                            int* __restrict__ list, unsigned long long* list_ctr,
                                                            float* __restrict__ width)
{
    constexpr int W = kEwListThreads / kWave;
    __shared__ int wsum[W];
    __shared__ unsigned long long block_base;
    const long long b0 = (long long)blockIdx.x * kEwListThreads;
    const long long i = b0 + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const long long nb = count - b0 < kEwListThreads ? count - b0 : kEwListThreads;
    for (long long q = threadIdx.x; q < nb * K; q += kEwListThreads) width[(first + b0) * K + q] = NAN;
    int nr = 0;
    if (i < count) {
        nr = n_ret[first + i];
        nr = nr < 0 ? 0 : (nr > K ? K : nr);
    }
    // prefix of nr over the wavefront, then over the block's wavefront totals
    int incl = nr;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        int t = lane < W ? wsum[lane] : 0;
        for (int off = 1; off < W; off <<= 1) {
            const int y = __shfl_up(t, off);
            if (lane >= off) t += y;
        }
        if (lane < W) wsum[lane] = t;
        if (lane == W - 1) block_base = t > 0 ? atomicAdd(list_ctr, (unsigned long long)t) : 0ull;
    }
    __syncthreads();
    const unsigned long long base = block_base + (unsigned long long)(w > 0 ? wsum[w - 1] : 0) + (incl - nr);
    const long long p = first + i;
    for (int k = 0; k < nr; ++k) list[base + k] = (int)(p * K + k);
}

// Residual sum, normal equations J'J (upper triangle 00 01 02 11 12 22) and J'r
// of the lane's lobe samples buf[q][lane] * inv, q in [L, R], x = q - kEwHalf,
// at (A, mu, s).
__device__ __forceinline__ float ew_pass(const float (*buf)[kWave], int lane, int L, int R, float inv, float A,
                                         float mu, float s, float H[6], float g[3])
{
    const float is = 1.0f / s;
    const float is2 = is * is;
    const float k2 = -0.5f * 1.4426950408889634f * is2;  // exp(-d^2 / (2 s^2)) = exp2(k2 d^2)
    float c = 0.0f;
    for (int q = 0; q < 6; ++q) H[q] = 0.0f;
    for (int q = 0; q < 3; ++q) g[q] = 0.0f;
    for (int q = L; q <= R; ++q) {
        const float y = buf[q][lane] * inv;
        const float d = (float)(q - kEwHalf) - mu;
        const float e = __builtin_amdgcn_exp2f(k2 * d * d);
        const float ae = A * e;
        const float r = y - ae;
        const float j1 = ae * d * is2;
        const float j2 = j1 * d * is;
        c = fmaf(r, r, c);
        H[0] = fmaf(e, e, H[0]);
        H[1] = fmaf(e, j1, H[1]);
        H[2] = fmaf(e, j2, H[2]);
        H[3] = fmaf(j1, j1, H[3]);
        H[4] = fmaf(j1, j2, H[4]);
        H[5] = fmaf(j2, j2, H[5]);
        g[0] = fmaf(e, r, g[0]);
        g[1] = fmaf(j1, r, g[1]);
        g[2] = fmaf(j2, r, g[2]);
    }
    return c;
}

__global__ __launch_bounds__(kWave) void k_ew_fit(const float* __restrict__ wf, int nb, int K, float bin_ns,
                                                  float s0, const int32_t* __restrict__ ret_bin,
                                                  const int* __restrict__ list,
                                                  const unsigned long long* __restrict__ list_ctr,
                                                  float* __restrict__ width)
{
    __shared__ float buf[kEwSpan][kWave];
    const int lane = threadIdx.x;
    const unsigned long long n = *list_ctr;
    const unsigned long long stride = (unsigned long long)gridDim.x * kWave;
    for (unsigned long long i = (unsigned long long)blockIdx.x * kWave + lane; __ballot(i < n);
         i += stride) {
        const bool mine = i < n;
        int e = 0, j = -1;
        if (mine) {
            e = list[i];
            j = ret_bin[e];
        }
        const long long row = (long long)(e / K) * nb;
        const bool ok = mine && j >= 0 && j < nb;
        // the bins around the return; +inf outside the waveform stops the lobe
        for (int q = 0; q < kEwSpan; ++q) {
            const int b = j - kEwHalf + q;
            buf[q][lane] = ok && b >= 0 && b < nb ? wf[row + b] : INFINITY;
        }
        int L = kEwHalf, R = kEwHalf;
        if (ok) {
            const float top = buf[kEwHalf][lane];
            while (L > 0 && buf[L - 1][lane] < buf[L][lane] && 1024.0f * buf[L - 1][lane] >= top) --L;
            while (R < kEwSpan - 1 && buf[R + 1][lane] < buf[R][lane] && 1024.0f * buf[R + 1][lane] >= top) ++R;
        }
        // the fit runs on the lobe divided by the return bin's value: least
        // squares is equivariant under that scaling (A scales, mu and s do not),
        // and faint echoes would otherwise underflow FP32 in the normal equations
        const int c = kEwHalf;
        const float peak = ok ? buf[c][lane] : 0.0f;
        const float inv = peak > 0.0f ? 1.0f / peak : 0.0f;
        float A = 1.0f, mu = 0.0f, s = s0;
        if (ok && peak > 0.0f && L <= c - 1 && R >= c + 1) {
            const float ym = buf[c - 1][lane] * inv, y0 = 1.0f, yp = buf[c + 1][lane] * inv;
            if (ym > 0.0f && yp > 0.0f) {
                const float lm = logf(ym), l0 = logf(y0), lp = logf(yp);
                const float c2 = lm - 2.0f * l0 + lp;
                if (c2 < 0.0f) {
                    const float s2 = -1.0f / c2;
                    mu = 0.5f * (lp - lm) * s2;
                    A = expf(l0 + mu * mu / (2.0f * s2));
                    s = sqrtf(s2);
                }
            }
        }
        const bool fit = ok && peak > 0.0f && R - L + 1 >= 3;
        if (fit) {
            float H[6], g[3];
            float cost = ew_pass(buf, lane, L, R, inv, A, mu, s, H, g);
            float lambda = 1e-3f;
            for (int it = 0; it < kEwIters; ++it) {
                // (H + lambda diag H) delta = g by Cramer's rule
                const float a = H[0] * (1.0f + lambda), b = H[1], cc = H[2], d = H[3] * (1.0f + lambda), ee = H[4],
                            f = H[5] * (1.0f + lambda);
                const float m0 = d * f - ee * ee, m1 = b * f - ee * cc, m2 = b * ee - d * cc;
                const float det = a * m0 - b * m1 + cc * m2;
                if (!(det != 0.0f) || !isfinite(det)) break;
                const float id = 1.0f / det;
                const float d0 = (g[0] * m0 - b * (g[1] * f - ee * g[2]) + cc * (g[1] * ee - d * g[2])) * id;
                const float d1 = (a * (g[1] * f - ee * g[2]) - g[0] * m1 + cc * (b * g[2] - g[1] * cc)) * id;
                const float d2 = (a * (d * g[2] - g[1] * ee) - b * (b * g[2] - g[1] * cc) + g[0] * m2) * id;
                const float tA = A + d0, tmu = mu + d1, ts = s + d2;
                const bool inside = fabsf(tmu) <= (float)(R - L) && fabsf(ts) <= 2.0f * (float)(R - L + 1);
                float Ht[6], gt[3];
                float ct = INFINITY;
                if (inside) ct = ew_pass(buf, lane, L, R, inv, tA, tmu, ts, Ht, gt);
                if (ct < cost) {
                    A = tA;
                    mu = tmu;
                    s = ts;
                    cost = ct;
                    for (int q = 0; q < 6; ++q) H[q] = Ht[q];
                    for (int q = 0; q < 3; ++q) g[q] = gt[q];
                    lambda *= 0.1f;
                } else {
                    lambda *= 10.0f;
                }
            }
        }
        if (mine) width[e] = fit && A > 0.0f && isfinite(s) && s != 0.0f ? fabsf(s) * bin_ns : NAN;
    }
}

inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_echo_width(const ScannerDev& sc, const float* wf, const int32_t* n_ret, const int32_t* ret_bin,
                             float s0_bins, long long first, long long count, int* list,
                             unsigned long long* list_ctr, float* width, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipError_t e = launch_fill_u64(list_ctr, 1, 0ull, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ew_list, dim3(grid_for(count, kEwListThreads)), dim3(kEwListThreads), 0, stream, n_ret, sc.K,
                       first, count, list, list_ctr, width);
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    // at most count * K returns; a grid of 8 wavefronts per compute unit strides over them
    const long long most = count * (long long)sc.K;
    long long blocks = (most + kWave - 1) / kWave;
    const long long cap = cus > 0 ? 8ll * cus : 2048ll;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_ew_fit, dim3((unsigned)blocks), dim3(kWave), 0, stream, wf, sc.n_bins, sc.K, sc.bin_ns,
                       s0_bins, ret_bin, list, list_ctr, width);
    return hipGetLastError();
}

}  // namespace vls
