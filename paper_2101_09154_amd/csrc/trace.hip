// The fused hot path on gfx950: subrays -> closest hit -> return power ->
// waveform -> returns, one wavefront per floor(64/S) pulses, one subray per lane.
//
// Subrays (Sec. 3.4, Fig. 6): the lane of subray k builds its direction in FP64
// from the pulse direction and a per-scanner table (cos a, sin a, cos phi,
// sin phi, weight) computed on the host:  d_k = cos a d + sin a (cos phi u +
// sin phi v), (u, v) the orthonormal basis of Duff et al. (2017).
//
// Closest hit (Sec. 3.4: a hit ends the subray; Sec. 5.1: minimum-distance
// intersection): the triangles a pulse's subrays can meet come from the cone
// pass (cone.hip); otherwise each subray walks the LBVH, near child first,
// boxes tested in FP32 against a per-ray padding that covers the rounding of
// the FP32 ray, so no box that holds the FP64 closest hit is culled.
// Triangles are tested in FP64 with the watertight test of Woop, Benthin &
// Wald (2013) (two-sided, inclusive edges, t > 0), so no subray slips through
// a shared edge and hit selection is the exact-arithmetic result up to FP64
// rounding; equal distances go to the lower triangle index.  A pulse alone in
// its wavefront first culls its candidates at staging and puts each survivor
// to its subrays' FP32 vote (edge_vote_coeffs), whose margins guarantee that
// only candidates no subray can be inside skip the FP64 test.  The traversal
// stack is a per-lane ring in LDS that spills its oldest entries to per-lane
// scratch when it is full.
//
// Power (Sec. 5.2, Eq. 7 with a Lambertian extended target):
//   P_k = P0 w_k (eta D^2 / 4) rho cos(theta) / R^2,  cos(theta) = |d_k . n|.
//
// Waveform (Sec. 3.4, Eq. 3 or a Gaussian pulse): the window starts t_pre
// before the pulse's first two-way travel time tau = 2R/c; lane l owns bins
// l + 64 m; each bin sums P_k p(t0 + j bin - tau_k) over the pulse's subrays,
// read from LDS, in fixed k order (deterministic).  Offsets are formed in FP64
// from the chunk's centre and split into two FP32 parts: the sums take the
// head, the attribution of returns both.  Only chunks of 64 bins that some
// subray's pulse support reaches are summed.
//
// Returns (Sec. 3.4 local maxima): bin j in [1, n-2] is a return if
// wf[j] > wf[j-1], wf[j] >= wf[j+1] and wf[j] >= max(abs, rel * max wf);
// neighbours come through lane shuffles, a ballot gives each return its slot,
// the first K in time order are kept, and each is attributed to the subray
// contributing most at its bin (lowest subray index on ties).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "vls_internal.h"
#include "device_common.h"
#include "voxels.h"

namespace vls {
namespace {

using namespace dev;

// A candidate triangle staged for the subrays of one pulse: its vertices
// translated to the pulse origin in FP64 (the first step of the watertight test,
// shared by all subrays of the pulse), its original index and its leaf.
struct CandRec {
    double a[3], b[3], c[3];
    int orig;
    int leaf;
};

// A candidate staged for a pulse alone in its wavefront (long candidate lists):
// its vertices as loaded (w: the original index, the leaf index, and the last
// component of the subrays' vote below), and the vote's other eight components.
// The FP64 translation to the pulse origin is redone, with the same operations
// as for a CandRec, only for candidates some subray may meet.
struct ChunkRec {
    float4 P0, P1, P2;
    float4 e0, e1;  // A0 B0 C0 A1 | B1 C1 A2 B2 (C2 in P2.w)
};
static_assert(sizeof(ChunkRec) == sizeof(CandRec), "a chunk slot is a staged slot");

// Per-wavefront LDS, used in turn by the two phases: the staged candidates of the
// wavefront's pulses (slot = pulse * staged_per_pulse + candidate) while tracing,
// then the subrays' waveform inputs (offset hi, offset lo, power, unused) per lane,
// followed by the kept returns of the two pulses of a paired wavefront (16 bytes
// per slot, VLS_MAX_RETURNS slots per pulse).
constexpr int kWaveInBytes = kWave * 16;
constexpr int kRetStageBytes = 2 * 16 * 16;
__host__ __device__ constexpr int wave_lds_bytes(int staged_slots)
{
    return staged_slots * (int)sizeof(CandRec) > kWaveInBytes + kRetStageBytes ? staged_slots * (int)sizeof(CandRec)
                                                                               : kWaveInBytes + kRetStageBytes;
}

__device__ __forceinline__ bool box_hit(const RayBox& r, float lx, float ly, float lz, float hx, float hy, float hz,
                                        float tcull, float& tn)
{
    float ax = fmaf(lx, r.inv[0], -r.oim[0]), bx = fmaf(hx, r.inv[0], -r.oip[0]);
    float ay = fmaf(ly, r.inv[1], -r.oim[1]), by = fmaf(hy, r.inv[1], -r.oip[1]);
    float az = fmaf(lz, r.inv[2], -r.oim[2]), bz = fmaf(hz, r.inv[2], -r.oip[2]);
    float n0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
    float f0 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tcull));
    tn = n0;
    return n0 <= f0;
}

struct Hit {
    double t;
    int leaf;
    int orig;
};

// Watertight ray/triangle test (Woop, Benthin & Wald 2013) in FP64, two-sided,
// inclusive edges, on vertices already translated to the ray origin: the
// triangle is sheared so the ray runs along +kz; the 2-D edge functions U, V, W
// are then evaluated from the same operands for both triangles of a shared edge,
// so no ray slips between them.  Returns t = T / det for a hit with t > 0, else
// a value that is not > 0 (NaN or <= 0).  tmax: the lane's closest distance so
// far; a hit provably beyond it is reported as a miss without the division
// (|T| above |det| tmax with a relative margin of 2^-40, far more than the
// rounding of the two products, means the quotient rounds above tmax, which
// the caller would reject; equal distances still take the division, since the
// caller breaks those ties by triangle index).
template <int KZ>
__device__ __forceinline__ double woop_t(const Ray& r, const double* a, const double* b, const double* c,
                                         double tmax)
{
#pragma clang fp contract(off)
    constexpr int KX = KZ == 2 ? 0 : KZ + 1;
    constexpr int KY = KX == 2 ? 0 : KX + 1;
    const double Az = a[KZ], Bz = b[KZ], Cz = c[KZ];
    const double Ax = a[KX] - r.Sx * Az, Ay = a[KY] - r.Sy * Az;
    const double Bx = b[KX] - r.Sx * Bz, By = b[KY] - r.Sy * Bz;
    const double Cx = c[KX] - r.Sx * Cz, Cy = c[KY] - r.Sy * Cz;
    const double U = Cx * By - Cy * Bx;
    const double V = Ax * Cy - Ay * Cx;
    const double W = Bx * Ay - By * Ax;
    const bool out = (U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0);
    const double det = U + V + W;
    // branches on the wavefront's votes: the scaled distance only where some
    // lane is inside the edges (most candidates miss every lane), the division
    // only where some lane can still hit closer
    double t = -1.0;
    const bool inside = !out && det != 0.0;
    if (__ballot(inside)) {
        const double T = U * (r.Sz * Az) + V * (r.Sz * Bz) + W * (r.Sz * Cz);
        const double lim = (fabs(det) * tmax) * (1.0 + 0x1p-40);
        const bool go = inside && !(fabs(T) > lim && lim >= 0x1p-1000);
        if (__ballot(go)) t = go ? T / det : -1.0;
    }
    return t;
}

// Closest-hit update: smaller t wins, equal t goes to the lower original index.
__device__ __forceinline__ bool closer(double t, int orig, const Hit& h)
{
    return t > 0.0 && (t < h.t || (t == h.t && orig < h.orig));
}

__device__ __forceinline__ void translate(const Ray& r, float4 P, double* v)
{
    v[0] = (double)P.x - r.O[0];
    v[1] = (double)P.y - r.O[1];
    v[2] = (double)P.z - r.O[2];
}

// Test of a triangle read from the leaf records (global memory); sets h.leaf.
__device__ __forceinline__ bool leaf_test(const Ray& r, const float4* __restrict__ tris, int li, Hit& h)
{
    const float4 P0 = tris[3 * li], P1 = tris[3 * li + 1], P2 = tris[3 * li + 2];
    double a[3], b[3], c[3];
    translate(r, P0, a);
    translate(r, P1, b);
    translate(r, P2, c);
    const double t = r.kz == 2 ? woop_t<2>(r, a, b, c, h.t)
                               : (r.kz == 1 ? woop_t<1>(r, a, b, c, h.t) : woop_t<0>(r, a, b, c, h.t));
    const int orig = __float_as_int(P0.w);
    if (!closer(t, orig, h)) return false;
    h.t = t;
    h.orig = orig;
    h.leaf = li;
    return true;
}

// The staged candidates [0, nc) of the lane's pulse (records from slot base on);
// KZ: the dominant axis of every active lane.  Returns the winning slot or -1.
template <int KZ>
__device__ __forceinline__ int cand_loop(const Ray& r, const CandRec* __restrict__ rec, int nc, Hit& h)
{
    int best = -1;
    for (int i = 0; i < nc; ++i) {
        const CandRec& c = rec[i];
        double a[3] = {c.a[0], c.a[1], c.a[2]}, b[3] = {c.b[0], c.b[1], c.b[2]}, e[3] = {c.c[0], c.c[1], c.c[2]};
        const double t = woop_t<KZ>(r, a, b, e, h.t);
        const int orig = c.orig;
        if (closer(t, orig, h)) {
            h.t = t;
            h.orig = orig;
            best = i;
        }
    }
    return best;
}

// Closest hit of one ray.  ring: this block's LDS ring, stride = blockDim.x.
// COUNT: also count internal-node visits and triangle tests.
template <bool COUNT>
__device__ __forceinline__ Hit traverse(const SceneDev& scene, const Ray& r, int* __restrict__ ring, int ring_mask,
                                        int& visits, int& tests)
{
    Hit h;
    h.t = INFINITY;
    h.leaf = -1;
    h.orig = 0x7fffffff;
    RayBox rb;
    setup_box(r, scene.bounds[12], rb);
    float tcull = INFINITY;
    const int stride = blockDim.x;
    int* my = ring + threadIdx.x;
    int spill[kMaxSpill];
    int sp = 0, nlow = 0;
    int node = scene.root;
    const float4* __restrict__ nodes = scene.nodes;
    // a traversal visits each of the 2n-1 nodes at most once; the cap and the
    // range checks only matter for a corrupted structure, which must not hang
    // or read out of bounds
    const int n_int = scene.n_tri - 1;
    int budget = 2 * scene.n_tri + 64;
    while (--budget > 0) {
        if (node >= n_int || ~node >= scene.n_tri) break;
        if (node >= 0) {
            if (COUNT) ++visits;
            const float4* nd = nodes + 4 * node;
            float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
            float tl, tr;
            bool hl = box_hit(rb, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tcull, tl);
            bool hr = box_hit(rb, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tcull, tr);
            int cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
            if (hl && hr) {
                int nearc = (tl <= tr) ? cl : cr;
                int farc = (tl <= tr) ? cr : cl;
                if (sp - nlow > ring_mask) {
                    // the host guarantees depth <= ring + kMaxSpill - 1; the guard keeps
                    // a violated guarantee from writing past the array
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
            if (COUNT) ++tests;
            if (leaf_test(r, scene.tris, ~node, h)) {
                // boxes beyond the closest hit so far cannot hold a closer one
                float tf = (float)h.t;
                if ((double)tf < h.t) tf = nextafterf(tf, INFINITY);
                tcull = tf;
            }
        }
        if (sp == 0) break;
        --sp;
        if (sp < nlow) {
            node = sp < kMaxSpill ? spill[sp] : -1;
            nlow = sp;
        } else {
            node = my[(sp & ring_mask) * stride];
        }
    }
    return h;
}

// Closest hits of the subrays of one pulse (the lanes with `on`), found by one
// walk of the wavefront over the four-wide records: the pulse's subrays are
// nearly parallel, so they share most of their path.  Each lane tests the
// children's boxes with its own padded FP32 ray and its own closest-hit
// distance; a child is entered when any lane's test passes, nearest first by
// the first lane's entry distance; every lane tests the leaves with its own
// FP64 watertight test.  Control flow and the stack are uniform: the stack sits
// in the wavefront's part of the LDS ring (entry e at word (e / 64) * stride +
// e % 64 of the wavefront's base), `cap` entries.  The host guarantees that
// 3 * ceil(depth / 2) <= cap.
template <bool COUNT>
__device__ __forceinline__ void packet_walk(const SceneDev& scene, const Ray& r, bool on, Hit& h,
                                            int* __restrict__ ring, int cap, int& visits, int& tests)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int stride = blockDim.x;
    int* st = ring + (threadIdx.x - lane);
    RayBox rb;
    setup_box(r, scene.bounds[12], rb);
    float tcull = INFINITY;
    const unsigned long long onm = __ballot(on);
    const int leader = __ffsll((long long)onm) - 1;
    const int n_int = scene.n_tri - 1;
    int node = scene.root;
    int sp = 0;
    for (int guard = 2 * scene.n_tri + 64; guard > 0; --guard) {
        if (node >= 0) {
            if (node >= n_int) break;  // only a corrupted structure gets here
            if (COUNT && on) ++visits;
            const float4* nd = scene.nodes4 + 8 * node;
            const float4 LX = nd[0], LY = nd[1], LZ = nd[2], HX = nd[3], HY = nd[4], HZ = nd[5], RF = nd[6];
            int rf[4] = {__float_as_int(RF.x), __float_as_int(RF.y), __float_as_int(RF.z), __float_as_int(RF.w)};
            float t[4];
            bool hit[4];
            hit[0] = on && rf[0] != kEmpty4 && box_hit(rb, LX.x, LY.x, LZ.x, HX.x, HY.x, HZ.x, tcull, t[0]);
            hit[1] = on && rf[1] != kEmpty4 && box_hit(rb, LX.y, LY.y, LZ.y, HX.y, HY.y, HZ.y, tcull, t[1]);
            hit[2] = on && rf[2] != kEmpty4 && box_hit(rb, LX.z, LY.z, LZ.z, HX.z, HY.z, HZ.z, tcull, t[2]);
            hit[3] = on && rf[3] != kEmpty4 && box_hit(rb, LX.w, LY.w, LZ.w, HX.w, HY.w, HZ.w, tcull, t[3]);
            // uniform keys: the leader's entry distance, 3e38 when only other
            // lanes enter the child, inf when none does
            float key[4];
            for (int i = 0; i < 4; ++i) {
                const float lt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hit[i] ? t[i] : 3e38f), leader));
                key[i] = __ballot(hit[i]) ? lt : INFINITY;
            }
#define VLS_CX(a, b)                                            \
    if (key[b] < key[a]) {                                      \
        const float kt = key[a]; key[a] = key[b]; key[b] = kt; \
        const int rr = rf[a]; rf[a] = rf[b]; rf[b] = rr;       \
    }
            VLS_CX(0, 1) VLS_CX(2, 3) VLS_CX(0, 2) VLS_CX(1, 3) VLS_CX(1, 2)
#undef VLS_CX
            for (int q = 3; q >= 1; --q) {
                if (key[q] < INFINITY && sp < cap) {
                    if (lane == 0) st[(sp >> 6) * stride + (sp & 63)] = rf[q];
                    ++sp;
                }
            }
            if (key[0] < INFINITY) {
                node = rf[0];
                continue;
            }
        } else {
            if (~node >= scene.n_tri) break;  // only a corrupted structure gets here
            if (on) {
                if (COUNT) ++tests;
                if (leaf_test(r, scene.tris, ~node, h)) {
                    // boxes beyond the closest hit so far cannot hold a closer one
                    float tf = (float)h.t;
                    if ((double)tf < h.t) tf = nextafterf(tf, INFINITY);
                    tcull = tf;
                }
            }
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(st[(sp >> 6) * stride + (sp & 63)]);
    }
}

// Incidence and power of the chosen triangle (Sec. 5.2, Eq. 7) in FP32, from
// its translated FP64 vertices: cos = |d . n| / |n|, P = C w rho f / R^2 with
// the surface response f = cos, or, for a scene with specular materials (Sec.
// 5.1), f = (1 - ks) cos + ks max(cos 2 theta, 0)^n: the mirror direction of a
// beam whose receiver sits at the emitter makes 2 theta with the way back.
__device__ __forceinline__ void shade(const Ray& r, const double* a, const double* b, const double* c, double t,
                                      float cw, float rho, const SceneDev& scene, int orig, float& cosang, float& P)
{
    const float e1x = (float)(b[0] - a[0]), e1y = (float)(b[1] - a[1]), e1z = (float)(b[2] - a[2]);
    const float e2x = (float)(c[0] - a[0]), e2y = (float)(c[1] - a[1]), e2z = (float)(c[2] - a[2]);
    const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const float nn = nx * nx + ny * ny + nz * nz;
    const float cs = nn > 0.0f ? fabsf(r.d32[0] * nx + r.d32[1] * ny + r.d32[2] * nz) / sqrtf(nn) : 0.0f;
    const float R = (float)t;
    cosang = cs;
    float f = cs;
    if (scene.spec_k) {
        const float ks = scene.spec_k[orig], n = scene.spec_n[orig];
        const float c2 = 2.0f * cs * cs - 1.0f;
        f = (1.0f - ks) * cs + ks * (c2 > 0.0f ? powf(c2, n) : 0.0f);
    }
    P = cw * rho * f / (R * R);
}

// Can any subray of a pulse meet this triangle (vertices translated to the
// pulse origin)?  In the pulse's basis (x = X.u, y = X.v, z = X.n) every subray
// direction lies in the square pyramid |x| <= k z, |y| <= k z with k the tangent
// of the largest subray angle, so a triangle whose three vertices all lie
// outside one of its four side planes, or all behind the origin, is met by no
// subray (its points are convex combinations of the vertices).  Only a cull
// test, in FP32: k is widened by 1e-5 relative and every comparison carries a
// margin of 1e-6 of the vertex's size (L1), several times the rounding of the
// vertex, the basis and the dot products, so a triangle some subray meets is
// never dropped.
struct CullBasis {
    float n[3], u[3], v[3];
    float k;
    float kc;  // >= 1 / cos(largest subray angle), with room for the FP32 axis
    float k2;  // k^2 (1 + 2^-18)
};

__device__ __forceinline__ CullBasis cull_basis(const Basis& Bs, double tan_max)
{
    CullBasis c;
    const double* n = Bs.n;
    const double sgn = copysign(1.0, n[2]);
    const double u[3] = {1.0 + sgn * n[0] * n[0] * Bs.a, sgn * Bs.b, -sgn * n[0]};
    const double v[3] = {Bs.b, sgn + n[1] * n[1] * Bs.a, -n[1]};
    for (int i = 0; i < 3; ++i) {
        c.n[i] = (float)n[i];
        c.u[i] = (float)u[i];
        c.v[i] = (float)v[i];
    }
    const double k = tan_max * (1.0 + 1e-5) + 1e-12;
    c.k = (float)k;
    c.kc = (float)(1.001 * sqrt(1.0 + k * k));
    c.k2 = (float)(k * k * (1.0 + 0x1p-18));
    return c;
}

__device__ __forceinline__ bool cone_may_hit(const float* A, const float* B, const float* C, const CullBasis& cb)
{
    bool px = true, nx = true, py = true, ny = true, bz = true;
    const float* X[3] = {A, B, C};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float w0 = X[i][0], w1 = X[i][1], w2 = X[i][2];
        const float z = fmaf(w0, cb.n[0], fmaf(w1, cb.n[1], w2 * cb.n[2]));
        const float x = fmaf(w0, cb.u[0], fmaf(w1, cb.u[1], w2 * cb.u[2]));
        const float y = fmaf(w0, cb.v[0], fmaf(w1, cb.v[1], w2 * cb.v[2]));
        const float m = 1e-6f * (fabsf(w0) + fabsf(w1) + fabsf(w2));
        const float kz = fmaf(cb.k, z, m);
        px = px && x > kz;
        nx = nx && -x > kz;
        py = py && y > kz;
        ny = ny && -y > kz;
        bz = bz && z < -m;
    }
    return !(px || nx || py || ny || bz);
}

__device__ __forceinline__ void stage_rec(CandRec& w, float4 P0, float4 P1, float4 P2, const double* o, int li)
{
    w.a[0] = (double)P0.x - o[0];
    w.a[1] = (double)P0.y - o[1];
    w.a[2] = (double)P0.z - o[2];
    w.b[0] = (double)P1.x - o[0];
    w.b[1] = (double)P1.y - o[1];
    w.b[2] = (double)P1.z - o[2];
    w.c[0] = (double)P2.x - o[0];
    w.c[1] = (double)P2.y - o[1];
    w.c[2] = (double)P2.z - o[2];
    w.orig = __float_as_int(P0.w);
    w.leaf = li;
}

// The subrays' vote on a candidate, a cheap pre-test of the watertight test's
// edge functions.  With the vertices a, b, c translated to the pulse origin,
// the watertight test's U, V, W for a subray of direction d are d.(c x b),
// d.(a x c) and d.(b x a) divided by one common factor, d's dominant component
// (the edge functions as scalar triple products, the Pluecker form of the edge
// test).  Since c x b = c x (b - c), each normal is formed in FP32 from one
// vertex relative to the origin and one edge of the triangle, n_i = p_i x e_i,
// so the FP32 products lose no digits to cancellation; its error is below
// 2^-22 |p_i|1 |e_i|1.  The normals are oriented so that a subray inside the
// edges has all three d.n_i >= 0: their sum d.N, N = (c - a) x (b - a), keeps
// one sign over the pulse's subrays when N.w - k |N|1 clears its margin (w the
// pulse axis, k the tangent of the largest subray angle); otherwise (the
// triangle's plane passes within the subrays' pyramid) every subray passes.
// Each normal then gets a margin m_i = 2^-17 |p_i|1 |e_i|1 + 2^-40 |p_i|1 |q_i|1
// (q_i the edge's other vertex; the FP64 rounding of U, V, W is below 2^-46 of
// that), folded in as m_i kc w with kc >= 1 / cos(largest subray angle), so that
// d.(n_i + m_i kc w) >= d.n_i + m_i for every subray.  Each margin-carrying
// normal is then taken to the pulse's basis (u, v, w): with d / (d.w) =
// x u + y v + w, (x, y) fixed per subray and x^2 + y^2 <= k^2, the vote of a
// subray on edge i is A_i x + B_i y + C_i >= 0, six fused multiply-adds for the
// three edges; its FP32 evaluation (basis, coefficients and x, y rounded to
// FP32) errs by less than 2^-20 |n_i|1, far inside the margin.  So a subray
// the watertight test finds inside the edges always votes yes, and a
// candidate no subray of the wavefront votes for would change no decision and
// is skipped.  A candidate for which some edge has C_i + k sqrt(A_i^2 + B_i^2)
// below -2^-20 (|A_i| + |B_i| + |C_i|) has every subray of the pulse outside
// that edge (the maximum of the vote over the disk of radius k), so no subray
// can vote for it and it is dropped at staging (the projected triangle and the
// beam's disk are separated along that edge's normal).
// t: the FP32 vertices relative to the origin; e: A0 B0 C0 A1 B1 C1 A2 B2 C2.
// Returns false for a candidate so dropped.
__device__ __forceinline__ bool edge_vote_coeffs(const float4& P0, const float4& P1, const float4& P2,
                                                 const float* ta, const float* tb, const float* tc,
                                                 const CullBasis& cb, float* e)
{
    float eb[3] = {P1.x - P2.x, P1.y - P2.y, P1.z - P2.z};  // b - c
    float ec[3] = {P2.x - P0.x, P2.y - P0.y, P2.z - P0.z};  // c - a
    float ea[3] = {P0.x - P1.x, P0.y - P1.y, P0.z - P1.z};  // a - b
    // N = (c - a) x (b - a), b - a = -ea
    const float Nx = fmaf(ec[2], ea[1], -(ec[1] * ea[2]));
    const float Ny = fmaf(ec[0], ea[2], -(ec[2] * ea[0]));
    const float Nz = fmaf(ec[1], ea[0], -(ec[0] * ea[1]));
    const float Nw = fmaf(Nx, cb.n[0], fmaf(Ny, cb.n[1], Nz * cb.n[2]));
    const float N1 = fabsf(Nx) + fabsf(Ny) + fabsf(Nz);
    const float la = fabsf(ta[0]) + fabsf(ta[1]) + fabsf(ta[2]);
    const float lb = fabsf(tb[0]) + fabsf(tb[1]) + fabsf(tb[2]);
    const float lc = fabsf(tc[0]) + fabsf(tc[1]) + fabsf(tc[2]);
    const float lea = fabsf(ea[0]) + fabsf(ea[1]) + fabsf(ea[2]);
    const float leb = fabsf(eb[0]) + fabsf(eb[1]) + fabsf(eb[2]);
    const float lec = fabsf(ec[0]) + fabsf(ec[1]) + fabsf(ec[2]);
    // one bound for the three edges: L = max |p|1, E = max |e|1
    const float L = fmaxf(la, fmaxf(lb, lc)), E = fmaxf(lea, fmaxf(leb, lec));
    const float mg = L * fmaf(0x1p-17f, E, 0x1p-40f * L);
    const float marg = fmaf(0x1p-18f * lec, lea, 0x1p-38f * 3.0f * L * L);
    const float spread = cb.k * N1;
    // beyond FP32's reach (also NaN): no orientation, a unit margin
    const bool fits = L * fmaxf(L, E) < 1e30f;
    float sg = Nw - spread > marg ? 1.0f : (-Nw - spread > marg ? -1.0f : 0.0f);
    sg = fits ? sg : 0.0f;
    const float mk = (fits ? fmaxf(mg, 0x1p-100f) : 1.0f) * cb.kc;
    // oriented normals n_i = p_i x (sg e_i) plus the folded margin; with sg = 0
    // only the margin is left and every subray votes yes
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        eb[j] *= sg;
        ec[j] *= sg;
        ea[j] *= sg;
    }
    const float* const pv[3] = {tc, ta, tb};
    const float* const ev[3] = {eb, ec, ea};
    bool may = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float* x = pv[i];
        const float* y = ev[i];
        const float n0 = fmaf(mk, cb.n[0], fmaf(x[1], y[2], -(x[2] * y[1])));
        const float n1 = fmaf(mk, cb.n[1], fmaf(x[2], y[0], -(x[0] * y[2])));
        const float n2 = fmaf(mk, cb.n[2], fmaf(x[0], y[1], -(x[1] * y[0])));
        const float A = fmaf(n0, cb.u[0], fmaf(n1, cb.u[1], n2 * cb.u[2]));
        const float B = fmaf(n0, cb.v[0], fmaf(n1, cb.v[1], n2 * cb.v[2]));
        const float C = fmaf(n0, cb.n[0], fmaf(n1, cb.n[1], n2 * cb.n[2]));
        e[3 * i] = A;
        e[3 * i + 1] = B;
        e[3 * i + 2] = C;
        // C + k sqrt(A^2 + B^2) < -eps  <=>  t = -C - eps > 0 and t^2 > k^2 (A^2 + B^2),
        // squared (k2 carries the squares' rounding): a product that flushes
        // to zero can only keep a candidate, never drop one wrongly
        const float t = fmaf(-0x1p-20f, fabsf(A) + fabsf(B) + fabsf(C), -C);
        may = may && !(t > 0.0f && t * t > cb.k2 * fmaf(A, A, B * B));
    }
    return may;
}

// Stage candidate li for the chunk loop: the FP32 vertices relative to the
// origin (for the culls and the vote; the watertight test redoes the FP64
// translation), the cull against the pulse's pyramid and the beam's disk, the
// vote's coefficients.  Returns whether the candidate may be met.
__device__ __forceinline__ bool stage_chunk(ChunkRec& w, float4 P0, float4 P1, float4 P2,
                                            const double* o, int li, bool b_ok, const CullBasis& cb)
{
    const float ta[3] = {(float)((double)P0.x - o[0]), (float)((double)P0.y - o[1]), (float)((double)P0.z - o[2])};
    const float tb[3] = {(float)((double)P1.x - o[0]), (float)((double)P1.y - o[1]), (float)((double)P1.z - o[2])};
    const float tc[3] = {(float)((double)P2.x - o[0]), (float)((double)P2.y - o[1]), (float)((double)P2.z - o[2])};
    float e[9];
    const bool may = edge_vote_coeffs(P0, P1, P2, ta, tb, tc, cb, e);
    w.P0 = P0;
    w.P1 = make_float4(P1.x, P1.y, P1.z, __int_as_float(li));
    w.P2 = make_float4(P2.x, P2.y, P2.z, e[8]);
    w.e0 = make_float4(e[0], e[1], e[2], e[3]);
    w.e1 = make_float4(e[4], e[5], e[6], e[7]);
    return !b_ok || (may && cone_may_hit(ta, tb, tc, cb));
}

// The chunk's records whose bits are set in `mask` (wave-uniform): the vote
// first ((x, y): the lane's subray in the pulse's basis, d / (d.w) = x u + y v
// + w), the watertight test only where some subray votes yes.  Returns the
// winning slot or -1.
template <int KZ>
__device__ __forceinline__ int chunk_loop(const Ray& r, float x, float y, const ChunkRec* __restrict__ rec,
                                          unsigned long long mask, Hit& h)
{
    int best = -1;
    for (; mask; mask &= mask - 1) {
        const int i = __ffsll((long long)mask) - 1;
        const float4 e0 = rec[i].e0, e1 = rec[i].e1;
        const float c2 = rec[i].P2.w;
        const float E0 = fmaf(e0.x, x, fmaf(e0.y, y, e0.z));
        const float E1 = fmaf(e0.w, x, fmaf(e1.x, y, e1.y));
        const float E2 = fmaf(e1.z, x, fmaf(e1.w, y, c2));
        if (__ballot(fminf(E0, fminf(E1, E2)) >= 0.0f)) {
            const ChunkRec& cr = rec[i];
            double a[3], b[3], c[3];
            translate(r, cr.P0, a);
            translate(r, cr.P1, b);
            translate(r, cr.P2, c);
            const double t = woop_t<KZ>(r, a, b, c, h.t);
            const int orig = __float_as_int(cr.P0.w);
            if (closer(t, orig, h)) {
                h.t = t;
                h.orig = orig;
                best = i;
            }
        }
    }
    return best;
}

__device__ __forceinline__ int chunk_loop_any(const Ray& r, float x, float y, const ChunkRec* rec,
                                              unsigned long long mask, Hit& h)
{
    // the mask is the wavefront's: keep it in scalar registers
    mask = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(mask >> 32)) << 32) |
           (unsigned)__builtin_amdgcn_readfirstlane((int)mask);
    if (r.kz == 2) return chunk_loop<2>(r, x, y, rec, mask, h);
    if (r.kz == 1) return chunk_loop<1>(r, x, y, rec, mask, h);
    return chunk_loop<0>(r, x, y, rec, mask, h);
}

// Trace one lane's subray: fills tri (original index or -1), R, cos, P.
// staged: the pulse's first min(nc, per) candidates sit in rec[q * per, ...)
// (per = staged_per_pulse); in a CHUNK launch only the n_kept of them that may
// meet one of its subrays, as ChunkRec slots [0, n_kept).
template <bool COUNT, bool CHUNK>
__device__ __forceinline__ void trace_lane(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                                           long long p, int k, int q, const Ray& r, const Basis& B, bool ray_ok,
                                           bool staged, int n_kept, CandRec* rec, int* ring, int ring_mask,
                                           int& tri, double& R, float& cosang, float& P, int& visits, int& tests)
{
    tri = -1;
    R = INFINITY;
    cosang = 0.0f;
    P = 0.0f;
    if (scene.n_tri <= 0 || !ray_ok) return;
    const double* pat = sc.pattern + 5 * k;
    Hit h;
    h.t = INFINITY;
    h.leaf = -1;
    h.orig = 0x7fffffff;
    const int nc = pulses.cand ? pulses.cand[p * (kCandMax + 1)] : -1;
    double a[3], b[3], c[3];
    if (CHUNK && nc >= 0 && staged) {
        // one pulse per wavefront: its first min(nc, 64) candidates were staged
        // by the whole wavefront, the n_kept of them that may meet a subray
        // packed in slots [0, n_kept); the rest are staged here in chunks of
        // S floor(64 / S), each triangle loaded by one subray lane (all of them
        // take this branch together, k = 0..S-1), culled, and marked in a
        // 64-bit mask
        ChunkRec* crec = reinterpret_cast<ChunkRec*>(rec);
        // the subray in the pulse's basis (from the subray table: d = cos a w +
        // sin a (cos phi u + sin phi v))
        const double ta = pat[1] / pat[0];
        const float x = (float)(ta * pat[2]), y = (float)(ta * pat[3]);
        const unsigned long long m0 = n_kept >= kWave ? ~0ull : ((1ull << n_kept) - 1ull);
        const int b0 = chunk_loop_any(r, x, y, crec, m0, h);
        int best_leaf = b0 >= 0 ? __float_as_int(crec[b0].P1.w) : -1;
        if (nc > kWave) {
            const int* cand = cand_ids(pulses.cand + p * (kCandMax + 1), nc, pulses.cand_long);
            const double* o = pulses.origins + 3 * p;
            const CullBasis cb = cull_basis(B, sc.tan_max);
            const int step = sc.S * (kWave / sc.S);
            for (int base = kWave; base < nc; base += step) {
                const int m = nc - base < step ? nc - base : step;
                wave_sync();  // the previous chunk has been read
                unsigned long long keep = 0;
                for (int j0 = 0; j0 < m; j0 += sc.S) {
                    const int j = j0 + k;
                    bool kp = false;
                    if (j < m) {
                        const int li = min(max(cand[base + j], 0), scene.n_tri - 1);
                        ChunkRec w;
                        kp = stage_chunk(w, scene.tris[3 * li], scene.tris[3 * li + 1], scene.tris[3 * li + 2], o, li,
                                         true, cb);
                        if (kp) crec[j] = w;
                    }
                    keep |= __ballot(kp) << j0;
                }
                wave_sync();
                const int b2 = chunk_loop_any(r, x, y, crec, keep, h);
                if (b2 >= 0) best_leaf = __float_as_int(crec[b2].P1.w);
            }
        }
        if (best_leaf < 0) return;
        // the winner's vertices come again from its leaf record (the same FP64
        // translation as in the test)
        h.leaf = best_leaf;
        translate(r, scene.tris[3 * h.leaf], a);
        translate(r, scene.tris[3 * h.leaf + 1], b);
        translate(r, scene.tris[3 * h.leaf + 2], c);
    } else if (nc >= 0 && staged) {
        // the cone pass found every triangle any subray of this pulse can hit;
        // the dominant axis is the same for the whole wavefront almost always, so
        // the test of the staged ones is specialised for it behind a uniform branch
        const int per = staged_per_pulse(sc.P_w);
        const CandRec* mine = rec + q * per;
        const int ns = nc < per ? nc : per;
        const int kz0 = __builtin_amdgcn_readfirstlane(r.kz);
        int best;
        if (__ballot(r.kz != kz0) == 0) {
            if (kz0 == 2) best = cand_loop<2>(r, mine, ns, h);
            else if (kz0 == 1) best = cand_loop<1>(r, mine, ns, h);
            else best = cand_loop<0>(r, mine, ns, h);
        } else {
            if (r.kz == 2) best = cand_loop<2>(r, mine, ns, h);
            else if (r.kz == 1) best = cand_loop<1>(r, mine, ns, h);
            else best = cand_loop<0>(r, mine, ns, h);
        }
        // candidates beyond the staged ones come from the leaf records
        const int* cand = cand_ids(pulses.cand + p * (kCandMax + 1), nc, pulses.cand_long);
        for (int i = ns; i < nc; ++i) leaf_test(r, scene.tris, cand[i], h);
        if (COUNT) tests += nc;
        if (h.leaf >= 0) {
            translate(r, scene.tris[3 * h.leaf], a);
            translate(r, scene.tris[3 * h.leaf + 1], b);
            translate(r, scene.tris[3 * h.leaf + 2], c);
        } else {
            if (best < 0) return;
            const CandRec& w = mine[best];
            for (int i = 0; i < 3; ++i) {
                a[i] = w.a[i];
                b[i] = w.b[i];
                c[i] = w.c[i];
            }
        }
    } else {
        if (nc >= 0 || nc == kWalked) {
            // the pulse's candidates, or the one leaf a packet walk found for
            // this subray (-1: none)
            const int* ids = pulses.cand + p * (kCandMax + 1) + 1;
            if (nc > kCandMax) ids = cand_ids(ids - 1, nc, pulses.cand_long);
            int cnt = nc;
            if (nc == kWalked) {
                cnt = 1;
                ids += k;
            }
            for (int i = 0; i < cnt; ++i) {
                const int li = ids[i];
                if (li >= 0 && li < scene.n_tri) leaf_test(r, scene.tris, li, h);
            }
            if (COUNT) tests += cnt;
        } else {
            h = traverse<COUNT>(scene, r, ring, ring_mask, visits, tests);
        }
        if (h.leaf < 0) return;
        translate(r, scene.tris[3 * h.leaf], a);
        translate(r, scene.tris[3 * h.leaf + 1], b);
        translate(r, scene.tris[3 * h.leaf + 2], c);
    }
    shade(r, a, b, c, h.t, (float)(sc.power_c * pat[4]), scene.refl[h.orig], scene, h.orig, cosang, P);
    tri = h.orig;
    R = h.t;
}

// Waveform rows are written once and not read back by the kernel: streaming
// (non-temporal) stores keep them from displacing the scene in the caches.
typedef float vf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void stream_store(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stream_zero4(float4* p)
{
    const vf4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    __builtin_nontemporal_store(z, reinterpret_cast<vf4*>(p));
}

// Contribution of one echo to a bin: offsets are taken from the centre bin jc of
// the bin's chunk, so x = (l - 32) bin (lane l) and the echo offset
// r = (tau - t0) - jc bin (FP64, split into FP32 hi + lo) are both small.  The
// waveform sums take s = x - hi: |r| stays within a chunk's reach (tens of ns),
// so dropping lo moves s by at most half an FP32 ulp of r (~1e-6 ns) and a bin's
// value by ~1e-6 relative at the pulse's flanks, a tenth of the waveform bound;
// the attribution of returns, which compares subrays at one bin, takes
// s = (x - hi) - lo with FP64 accuracy.
__device__ __forceinline__ void echo_offset(const ScannerDev& sc, double rel, int jc, float& hi, float& lo)
{
    const double r = rel - (double)jc * sc.bin_d;
    hi = (float)r;
    lo = (float)(r - (double)hi);
}

template <int SHAPE>
__device__ __forceinline__ float echo_value(const ScannerDev& sc, float x, float hi, float lo, float pw)
{
    return pw * pulse_shape<SHAPE>(sc, (x - hi) - lo);
}

// Waveform and/or returns of one pulse whose subrays are lanes [k0, k0 + S).
// Each lane passes its own subray (tau = 2R/c, power, triangle; tri < 0: miss).
// COMPUTE: synthesise wf from the subrays (else load wf and t0 from `out`).
// RET: detect returns.  attrib: subray data present for return attribution.
//
// A synthesised waveform is non-zero only on the support [jl, jh] of its echoes,
// so it is computed as nch chunks of 64 bins starting at jb = jl (lane l of chunk
// c owns bin jb + 64 c + l); a loaded one as the aligned chunks of the whole row.
// Bins outside the chunks are zero.
// PACK: each chunk sums only the echoes that reach it (one pulse per wavefront,
// where echoes spread over several chunks; elsewhere the plain loop over all
// subrays is kept, which measured faster there).  The echoes left out add
// exactly zero to every bin of the chunk, so both loops give the same bits.
template <int MAXCH, bool COMPUTE, bool RET, int SHAPE, bool PACK = false>
__device__ __forceinline__ void pulse_phase(const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                                            long long p, int k0, float4* sub, bool attrib, double my_tau,
                                            float my_pw, int my_tri)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int S = sc.S, nb = sc.n_bins, K = sc.K;
    const bool sub_lane = lane >= k0 && lane < k0 + S;
    const bool mine = sub_lane && my_tri >= 0;
    double t0, tmin = INFINITY;
    bool any;
    if (COMPUTE || attrib) {
        tmin = wave_min_d(mine ? my_tau : INFINITY);
        any = tmin < INFINITY;
        if (COMPUTE) {
            if (pulses.t0_in) t0 = pulses.t0_in[p];
            else t0 = any ? tmin - sc.t_pre : (double)NAN;
        } else {
            t0 = out.t0[p];
        }
    } else {
        t0 = out.t0[p];
        any = true;
    }
    const bool have = any && !isnan(t0);
    const double rel = my_tau - t0;  // used on `mine` lanes only
    const float x = (float)((double)(lane - 32) * sc.bin_d);
    int jb = 0, nch = 0;
    if (!COMPUTE) {
        nch = (nb + kWave - 1) / kWave;
    } else if (have) {
        // support of the echoes in bins, widened by one bin against rounding: it
        // starts at the earliest echo (tmin) and ends at the latest (the largest
        // offset); the window starts there, rounded down to a multiple of 4 bins
        // (the bins it adds are computed like the others)
        const float lo = (float)(tmin - t0);
        const float hi = wave_max_f(mine ? (float)rel : -INFINITY);
        const int jl = (int)fminf(fmaxf(floorf((lo - sc.cut_lo) * sc.inv_bin) - 1.0f, 0.0f), 1e9f);
        const int jh = (int)fminf(fmaxf(ceilf((hi + sc.cut_hi) * sc.inv_bin) + 1.0f, -1.0f), (float)(nb - 1));
        if (jl <= jh) {
            jb = jl & ~3;
            nch = ((jh - jb) >> 6) + 1;
        }
    }
    float wf[MAXCH];
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) wf[c] = 0.0f;
    // an echo reaches a chunk if its pulse is non-zero at one of the chunk's
    // bins, whose offsets from the centre lie within [-33, 32] bins (one bin of
    // slack).  pulse_shape is exactly zero where its exp2 argument is below
    // -160 (the result is far below the smallest FP32 subnormal): the Gaussian
    // beyond |s| = sqrt(160 / -neg_k), Eq. 3 at s <= 0 and beyond s = 160 /
    // (-neg_k inv_tau); widened by 1e-3 against the FP32 rounding of s and of
    // the exponent, an echo outside [-33 bin - z_pos, 32 bin + z_neg] adds
    // exactly zero to each of the chunk's bins
    const float z_pos = 1.001f * (SHAPE == 0 ? sqrtf(-160.0f / sc.neg_k) : -160.0f / (sc.neg_k * sc.inv_tau));
    const float z_neg = SHAPE == 0 ? z_pos : 0.0f;
    const float reach_lo = -33.0f * sc.bin_ns - z_pos, reach_hi = 32.0f * sc.bin_ns + z_neg;
    if (COMPUTE) {
#pragma unroll
        for (int c = 0; c < MAXCH; ++c) {
            if (c >= nch) continue;
            float acc = 0.0f;
            if (PACK) {
                // the echoes that reach the chunk, packed in subray order (missed
                // subrays add nothing and are left out too)
                float hi = 0.0f, lo = 0.0f;
                if (mine) echo_offset(sc, rel, jb + c * kWave + 32, hi, lo);
                const bool reach = mine && hi >= reach_lo && hi <= reach_hi;
                const unsigned long long rm = __ballot(reach);
                if (reach) sub[lanes_below(rm)] = make_float4(hi, 0.0f, my_pw, 0.0f);
                const int nr = __popcll(rm);
                wave_sync();
#pragma unroll 4
                for (int kk = 0; kk < nr; ++kk) {
                    const float4 u = sub[kk];
                    acc = fmaf(u.z, pulse_shape<SHAPE>(sc, x - u.x), acc);
                }
            } else {
                if (sub_lane) {
                    // a missed subray carries power 0 and offset 0: it adds exactly 0
                    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (mine) {
                        echo_offset(sc, rel, jb + c * kWave + 32, v.x, v.y);
                        v.z = my_pw;
                    }
                    sub[lane] = v;
                }
                wave_sync();
#pragma unroll 4
                for (int kk = 0; kk < S; ++kk) {
                    const float4 u = sub[k0 + kk];
                    acc = fmaf(u.z, pulse_shape<SHAPE>(sc, x - u.x), acc);
                }
            }
            wf[c] = jb + c * kWave + lane < nb ? acc : 0.0f;
            wave_sync();
        }
        if (out.wf) {
            float* row = out.wf + p * nb;
            const int jend = jb + nch * kWave;
            if ((nb & 3) == 0 && (reinterpret_cast<unsigned long long>(out.wf) & 15) == 0) {
                // zeros outside the chunks, four bins per lane (jb and jend are
                // multiples of 4, and the row start is 16-byte aligned)
                float4* row4 = reinterpret_cast<float4*>(row);
#pragma unroll
                for (int m = 0; m < (MAXCH + 3) / 4; ++m) {
                    const int g = m * kWave + lane, j = 4 * g;
                    if (j < nb && (j < jb || j >= jend)) stream_zero4(&row4[g]);
                }
            } else {
#pragma unroll
                for (int m = 0; m < MAXCH; ++m) {
                    const int j = m * kWave + lane;
                    if (j < nb && (j < jb || j >= jend)) stream_store(&row[j], 0.0f);
                }
            }
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
                const int j = jb + c * kWave + lane;
                if (c < nch && j < nb) stream_store(&row[j], wf[c]);
            }
        }
        if (lane == 0 && out.t0) out.t0[p] = t0;
    } else {
#pragma unroll
        for (int c = 0; c < MAXCH; ++c) {
            int j = c * kWave + lane;
            if (j < nb) wf[c] = out.wf[p * nb + j];
        }
    }
    if (!RET) return;
    int count = 0;
    if (have && nch > 0) {
        float m = 0.0f;
#pragma unroll
        for (int c = 0; c < MAXCH; ++c)
            if (c < nch) m = fmaxf(m, wf[c]);
        m = wave_max_f(m);
        float thr = fmaxf((float)sc.thr_abs, (float)(sc.thr_rel * (double)m));
#pragma unroll
        for (int c = 0; c < MAXCH; ++c) {
            if (c >= nch || count >= K) continue;
            float v = wf[c];
            // neighbours: lane shifts, with the adjacent chunk's edge lane at the
            // chunk ends; beyond the first and last chunk the waveform is zero
            float prev = c > 0 ? lane_read_f(wf[c > 0 ? c - 1 : 0], 63) : 0.0f;
            float next = c + 1 < MAXCH && c + 1 < nch ? lane_read_f(wf[c + 1 < MAXCH ? c + 1 : c], 0) : 0.0f;
            float left = lane_prev_f(v, prev);
            float right = lane_next_f(v, next);
            const int j = jb + c * kWave + lane;
            bool cand = j >= 1 && j <= nb - 2 && v > left && v >= right && v >= thr;
            unsigned long long mk = __ballot(cand);
            int rt = -1;
            if (attrib && out.ret_tri && mk) {
                // each kept return goes to the subray contributing most at its bin
                // (lowest subray index on ties); subray lanes evaluate their own echo
                float hi = 0.0f, lo = 0.0f;
                if (mine) echo_offset(sc, rel, jb + c * kWave + 32, hi, lo);
                unsigned long long todo = mk;
                for (int s = count; todo && s < K; ++s) {
                    const int b = __ffsll((long long)todo) - 1;
                    todo &= todo - 1;
                    const float xb = (float)((double)(b - 32) * sc.bin_d);
                    const float val = mine ? echo_value<SHAPE>(sc, xb, hi, lo, my_pw) : -1.0f;
                    const float best = wave_max_f(val);
                    const unsigned long long w = __ballot(mine && val == best);
                    int t = -1;
                    if (w) t = __builtin_amdgcn_readlane(my_tri, __ffsll((long long)w) - 1);
                    if (lane == b) rt = t;
                }
            }
            int slot = count + (int)lanes_below(mk);
            if (cand && slot < K) {
                long long o = p * K + slot;
                out.ret_range[o] = (float)(0.5 * kCmPerNs * (t0 + (double)j * sc.bin_d - sc.s_peak));
                out.ret_amp[o] = v;
                out.ret_bin[o] = j;
                if (out.ret_tri) out.ret_tri[o] = rt;
            }
            count += __popcll(mk);
        }
    }
    int nret = count < K ? count : K;
    if (lane >= nret && lane < K) {
        long long o = p * K + lane;
        out.ret_range[o] = 0.0f;
        out.ret_amp[o] = 0.0f;
        out.ret_bin[o] = -1;
        if (out.ret_tri) out.ret_tri[o] = -1;
    }
    if (lane == 0) out.n_ret[p] = nret;
}

// Waveform and returns of the two pulses of a wavefront at once, pulse h in
// lanes 32 h .. 32 h + 31 (its subray k in lane 32 h + k, S <= 32), with the same
// results, bit for bit, as pulse_phase on each in turn: the same chunks of 64
// bins from the same window start, each lane holding bins jb + 64 c + l and
// jb + 64 c + 32 + l of its pulse (l = lane & 31), the same offsets from the
// chunk's centre bin and the same sums in subray order.  Reductions run over
// half wavefronts, so the two pulses share every reduction, neighbour exchange
// and ballot, and each subray record read from LDS serves two bins.
template <int MAXCH, int SHAPE>
__device__ __forceinline__ void pulse_pair(const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                                           long long first, float4* sub, double my_tau, float my_pw, int my_tri,
                                           bool sub_lane)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int h = lane >> 5, l = lane & 31, hb = lane & 32;
    const int S = sc.S, nb = sc.n_bins, K = sc.K;
    const long long p = first + h;
    const bool mine = sub_lane && my_tri >= 0;
    const double tmin = half_min_d(mine ? my_tau : INFINITY);
    const bool any = tmin < INFINITY;
    double t0;
    if (pulses.t0_in) t0 = pulses.t0_in[p];
    else t0 = any ? tmin - sc.t_pre : (double)NAN;
    const bool have = any && !isnan(t0);
    const double rel = my_tau - t0;  // used on `mine` lanes only
    const float x0 = (float)((double)(l - 32) * sc.bin_d), x1 = (float)((double)l * sc.bin_d);
    int jb = 0, nch = 0;
    {
        const float lo = (float)(tmin - t0);
        const float hi = half_max_f(mine ? (float)rel : -INFINITY);
        if (have) {
            const int jl = (int)fminf(fmaxf(floorf((lo - sc.cut_lo) * sc.inv_bin) - 1.0f, 0.0f), 1e9f);
            const int jh = (int)fminf(fmaxf(ceilf((hi + sc.cut_hi) * sc.inv_bin) + 1.0f, -1.0f), (float)(nb - 1));
            if (jl <= jh) {
                jb = jl & ~3;
                nch = ((jh - jb) >> 6) + 1;
            }
        }
    }
    const int nch_max = max(__builtin_amdgcn_readlane(nch, 0), __builtin_amdgcn_readlane(nch, 32));
    float wa[MAXCH], wb[MAXCH];
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
        wa[c] = 0.0f;
        wb[c] = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
        if (c >= nch_max) continue;
        if (sub_lane) {
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (mine && c < nch) {
                echo_offset(sc, rel, jb + c * kWave + 32, v.x, v.y);
                v.z = my_pw;
            }
            sub[lane] = v;
        }
        wave_sync();
        float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll 4
        for (int kk = 0; kk < S; ++kk) {
            const float4 u = sub[hb + kk];
            acc0 = fmaf(u.z, pulse_shape<SHAPE>(sc, x0 - u.x), acc0);
            acc1 = fmaf(u.z, pulse_shape<SHAPE>(sc, x1 - u.x), acc1);
        }
        const int j0 = jb + c * kWave + l;
        if (c < nch) {
            wa[c] = j0 < nb ? acc0 : 0.0f;
            wb[c] = j0 + 32 < nb ? acc1 : 0.0f;
        }
        wave_sync();
    }
    if (out.wf) {
        float* row = out.wf + p * nb;
        const int jend = jb + nch * kWave;
        if ((nb & 3) == 0 && (reinterpret_cast<unsigned long long>(out.wf) & 15) == 0) {
            float4* row4 = reinterpret_cast<float4*>(row);
#pragma unroll
            for (int m = 0; m < (MAXCH + 1) / 2; ++m) {
                const int g = m * 32 + l, j = 4 * g;
                if (j < nb && (j < jb || j >= jend)) stream_zero4(&row4[g]);
            }
        } else {
#pragma unroll
            for (int m = 0; m < 2 * MAXCH; ++m) {
                const int j = m * 32 + l;
                if (j < nb && (j < jb || j >= jend)) stream_store(&row[j], 0.0f);
            }
        }
#pragma unroll
        for (int c = 0; c < MAXCH; ++c) {
            const int j = jb + c * kWave + l;
            if (c < nch && j < nb) stream_store(&row[j], wa[c]);
            if (c < nch && j + 32 < nb) stream_store(&row[j + 32], wb[c]);
        }
    }
    if (l == 0 && out.t0) out.t0[p] = t0;
    // returns (Sec. 3.4 local maxima), as in pulse_phase, per half.  The kept
    // returns go to LDS slots first (bin order, as found), then lanes l < K of
    // each half write the pulse's K output slots once, zeros past its count.
    float m = 0.0f;
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
        if (c >= nch_max) break;
        m = fmaxf(m, fmaxf(wa[c], wb[c]));
    }
    m = half_max_f(m);
    const float thr = fmaxf((float)sc.thr_abs, (float)(sc.thr_rel * (double)m));
    float4* ret_st = reinterpret_cast<float4*>(reinterpret_cast<unsigned char*>(sub) + kWaveInBytes) + 16 * h;
    // kept so far in each half (wave-uniform values)
    int cnt_lo = 0, cnt_hi = 0;
    const unsigned long long lo_lanes = 0x00000000FFFFFFFFull;
    float hi_off = 0.0f, lo_off = 0.0f;
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
        if (c >= nch_max) break;
        if (cnt_lo >= K && cnt_hi >= K) break;
        const int count = h ? cnt_hi : cnt_lo;
        const bool act = have && c < nch && count < K;
        const float v0 = wa[c], v1 = wb[c];
        // neighbours in bin order: bin jb + 64 c + l has v0 of lane l - 1 and l + 1,
        // the last bin of the previous chunk at l = 0 and v1 of l = 0 at l = 31;
        // bin jb + 64 c + 32 + l likewise, with v0 of l = 31 at l = 0 and the first
        // bin of the next chunk at l = 31 (zero beyond the pulse's chunks)
        float left0 = lane_prev_f(v0, 0.0f), right0 = lane_next_f(v0, 0.0f);
        float left1 = lane_prev_f(v1, 0.0f), right1 = lane_next_f(v1, 0.0f);
        if (l == 0) {
            left0 = c > 0 ? __int_as_float(half_pick_i(__float_as_int(wb[c > 0 ? c - 1 : 0]))) : 0.0f;
            left1 = __int_as_float(half_pick_i(__float_as_int(v0)));
        }
        if (l == 31) {
            right0 = __int_as_float(h ? __builtin_amdgcn_readlane(__float_as_int(v1), 32)
                                      : __builtin_amdgcn_readlane(__float_as_int(v1), 0));
            float f = 0.0f;
            if (c + 1 < MAXCH && c + 1 < nch_max) {
                const int wn = __float_as_int(wa[c + 1 < MAXCH ? c + 1 : c]);
                f = __int_as_float(h ? __builtin_amdgcn_readlane(wn, 32) : __builtin_amdgcn_readlane(wn, 0));
            }
            right1 = c + 1 < nch ? f : 0.0f;
        }
        const int j0 = jb + c * kWave + l, j1 = j0 + 32;
        const bool cand0 = act && (unsigned)(j0 - 1) <= (unsigned)(nb - 3) && v0 > left0 && v0 >= right0 && v0 >= thr;
        const bool cand1 = act && (unsigned)(j1 - 1) <= (unsigned)(nb - 3) && v1 > left1 && v1 >= right1 && v1 >= thr;
        const unsigned long long mk0 = __ballot(cand0), mk1 = __ballot(cand1);
        if ((mk0 | mk1) == 0) continue;
        // per half: candidates of the first and second 32 bins (wave-uniform)
        const unsigned a_lo = (unsigned)mk0, b_lo = (unsigned)mk1;
        const unsigned a_hi = (unsigned)(mk0 >> 32), b_hi = (unsigned)(mk1 >> 32);
        const int n_lo = __popc(a_lo) + __popc(b_lo), n_hi = __popc(a_hi) + __popc(b_hi);
        const int take_lo = max(0, min(n_lo, K - cnt_lo)), take_hi = max(0, min(n_hi, K - cnt_hi));
        int rt0 = -1, rt1 = -1;
        if (out.ret_tri) {
            // each kept return goes to the subray contributing most at its bin
            // (lowest subray index on ties): both halves walk their returns in
            // bin order together, one half-wavefront maximum per step
            if (mine) echo_offset(sc, rel, jb + c * kWave + 32, hi_off, lo_off);
            const int steps = max(take_lo, take_hi);
            unsigned ra_lo = a_lo, rb_lo = b_lo, ra_hi = a_hi, rb_hi = b_hi;
            for (int s2 = 0; s2 < steps; ++s2) {
                // each half's next return: position in the chunk (0..63), or -1
                int bl = -1, bh = -1;
                if (s2 < take_lo) {
                    if (ra_lo) {
                        bl = __ffs((int)ra_lo) - 1;
                        ra_lo &= ra_lo - 1;
                    } else {
                        bl = 32 + __ffs((int)rb_lo) - 1;
                        rb_lo &= rb_lo - 1;
                    }
                }
                if (s2 < take_hi) {
                    if (ra_hi) {
                        bh = __ffs((int)ra_hi) - 1;
                        ra_hi &= ra_hi - 1;
                    } else {
                        bh = 32 + __ffs((int)rb_hi) - 1;
                        rb_hi &= rb_hi - 1;
                    }
                }
                const int b = h ? bh : bl;
                const float xb = (float)((double)(b - 32) * sc.bin_d);
                const float val = mine && b >= 0 ? echo_value<SHAPE>(sc, xb, hi_off, lo_off, my_pw) : -1.0f;
                const float best = half_max_f(val);
                // each half's winner: the lowest of its lanes at the maximum
                // (read with lane numbers that are the same for the whole wavefront)
                const unsigned long long w = __ballot(mine && b >= 0 && val == best);
                const unsigned w_lo = (unsigned)w, w_hi = (unsigned)(w >> 32);
                const int t_lo = w_lo ? __builtin_amdgcn_readlane(my_tri, __ffs((int)w_lo) - 1) : -1;
                const int t_hi = w_hi ? __builtin_amdgcn_readlane(my_tri, 32 + __ffs((int)w_hi) - 1) : -1;
                const int t = h ? t_hi : t_lo;
                if (b >= 0 && l == (b & 31)) {
                    if (b < 32) rt0 = t;
                    else rt1 = t;
                }
            }
        }
        // slots: this half's count, then the first 32 bins' candidates below the
        // lane, then the second 32 bins' below it
        const unsigned a_h = h ? a_hi : a_lo, b_h = h ? b_hi : b_lo;
        const unsigned below = (1u << l) - 1u;
        const int slot0 = count + __popc(a_h & below);
        const int slot1 = count + __popc(a_h) + __popc(b_h & below);
        if (cand0 && slot0 < K) {
            const float rg = (float)(0.5 * kCmPerNs * (t0 + (double)j0 * sc.bin_d - sc.s_peak));
            ret_st[slot0] = make_float4(rg, v0, __int_as_float(j0), __int_as_float(rt0));
        }
        if (cand1 && slot1 < K) {
            const float rg = (float)(0.5 * kCmPerNs * (t0 + (double)j1 * sc.bin_d - sc.s_peak));
            ret_st[slot1] = make_float4(rg, v1, __int_as_float(j1), __int_as_float(rt1));
        }
        cnt_lo += n_lo;
        cnt_hi += n_hi;
    }
    wave_sync();
    const int nret = min(h ? cnt_hi : cnt_lo, K);
    if (l < K) {
        float4 r = make_float4(0.0f, 0.0f, __int_as_float(-1), __int_as_float(-1));
        if (l < nret) r = ret_st[l];
        const long long o = p * K + l;
        out.ret_range[o] = r.x;
        out.ret_amp[o] = r.y;
        out.ret_bin[o] = __float_as_int(r.z);
        if (out.ret_tri) out.ret_tri[o] = __float_as_int(r.w);
    }
    if (l == 0) out.n_ret[p] = nret;
}

// One wavefront: pulses [first, first + npw) of one scanner.
// MODE 0: trace only.  MODE 1: trace + waveform + returns (fused).
// MODE 2: trace only, adding subrays / node visits / triangle tests to out.counts.
// CHUNK: a launch for a scanner with one pulse per wavefront, which stages long
// candidate lists in chunks (kept out of the other launches' code).
template <int MAXCH, int MODE, bool CHUNK, bool VOX>
__device__ __forceinline__ void process_wave(const SceneDev& scene, const ScannerDev& sc,
                                             const PulsesDev& pulses, const OutDev& out, long long first, int npw,
                                             int* ring, int ring_mask, unsigned char* wl)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int S = sc.S;
    // two pulses per wavefront in the fused launch: pulse h's subrays in lanes
    // 32 h + k, so that its waveform phase runs on half a wavefront (pulse_pair)
    const bool pair = MODE == 1 && !CHUNK && sc.P_w == 2 && npw == 2;
    const int pl = pair ? lane >> 5 : lane / S;
    const int k = pair ? lane & 31 : lane - pl * S;
    const bool active = pl < npw && k < S;
    // stage the first candidate triangles of up to 4 pulses, one per lane (64 for
    // one pulse per wavefront, else 16 per pulse), translated to their pulse's
    // origin
    // The loads are issued first and the subray setup runs while they are in
    // flight: the count and the ids share a row, and the record loads use an id
    // clamped into range, so they need not wait for the count.
    CandRec* rec = reinterpret_cast<CandRec*>(wl);
    const bool staged = pulses.cand && sc.P_w <= 4;
    // staged_per_pulse is 64 or 16: a shift, not a division
    const int per_shift = staged && sc.P_w == 1 ? 6 : 4;
    const int sq = lane >> per_shift, sc16 = lane & ((1 << per_shift) - 1);
    int nq = -1, li = 0;
    float4 P0, P1, P2;
    if (staged && sq < npw && scene.n_tri > 0) {
        const int* row = pulses.cand + (first + sq) * (kCandMax + 1);
        nq = row[0];
        int id = row[1 + sc16];  // loaded with the count; a long list's ids come after it
        if (nq > kCandMax && sc16 < nq) id = cand_ids(row, nq, pulses.cand_long)[sc16];
        li = min(max(id, 0), scene.n_tri - 1);
        P0 = scene.tris[3 * li];
        P1 = scene.tris[3 * li + 1];
        P2 = scene.tris[3 * li + 2];
    }
    Ray r;
    // the pulse's basis comes from the cone pass when it ran (same values)
    // (one pulse per wavefront: every lane loads it, the staging lanes beyond
    // the subrays test candidates against it)
    Basis B;
    const long long pb = CHUNK ? first : first + pl;
    const bool b_ok = (CHUNK || active) && (pulses.basis ? load_basis(pulses.basis + 5 * pb, B)
                                                         : pulse_basis(pulses.dirs + 3 * pb, B));
    const bool ray_ok = active && b_ok && setup_ray_b(pulses.origins + 3 * (first + pl), B, sc.pattern + 5 * k, r);
    // With one pulse per wavefront (long candidate lists), the staged
    // candidates that may meet one of its subrays, packed in list order (a
    // pulse without a valid direction keeps all: its subrays trace nothing);
    // with several, all of them (short lists, where the test costs more than
    // it saves).
    int n_kept = 0;
    if (staged) {
        if (CHUNK) {
            ChunkRec w;
            bool keep = false;
            if (sc16 < nq)
                keep = stage_chunk(w, P0, P1, P2, pulses.origins + 3 * (first + sq), li, b_ok,
                                   cull_basis(B, sc.tan_max));
            const unsigned long long kept = __ballot(keep);
            if (keep) reinterpret_cast<ChunkRec*>(wl)[lanes_below(kept)] = w;
            n_kept = __popcll(kept);
        } else if (sc16 < nq) {
            stage_rec(rec[lane], P0, P1, P2, pulses.origins + 3 * (first + sq), li);
        }
        wave_sync();
    }
    int tri = -1;
    double R = INFINITY;
    float cs = 0.0f, P = 0.0f;
    int visits = 0, tests = 0;
    if (active) {
        long long p = first + pl;
        trace_lane<MODE == 2, CHUNK>(scene, sc, pulses, p, k, pl, r, B, ray_ok, staged, n_kept, rec, ring, ring_mask,
                                     tri, R, cs, P,
                              visits, tests);
        if (VOX && ray_ok) {
            // a voxel that stops the subray before its closest triangle takes the
            // echo: id n_tri + voxel, cos 1, power by Eq. 7 (proportionality as
            // equality): P = power_c w sigma / (pi beta^2 R^4)
            double tv, sg;
            const uint64_t c0 = ((uint64_t)p * kWave + (uint64_t)k) * (uint64_t)scene.vox.n_vox;
            const long long vi = voxel_stop(scene.vox, r.O, r.D, tri >= 0 ? R : (double)INFINITY, c0, tv, sg);
            if (vi >= 0) {
                tri = scene.n_tri + (int)vi;
                R = tv;
                cs = 1.0f;
                const double R2 = tv * tv;
                P = (float)(sc.vox_c * sc.pattern[5 * k + 4] * sg / (R2 * R2));
            }
        }
        long long o = p * out.sub_stride + k;
        if (out.sub_tri) out.sub_tri[o] = tri;
        if (out.sub_range) out.sub_range[o] = R;
        if (out.sub_cos) out.sub_cos[o] = cs;
        if (out.sub_power) out.sub_power[o] = P;
    }
    if (MODE == 2) {
        unsigned long long a = active ? 1ull : 0ull, v = (unsigned long long)visits, t = (unsigned long long)tests;
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            v += __shfl_xor(v, o);
            t += __shfl_xor(t, o);
        }
        if (lane == 0) {
            atomicAdd(out.counts, a);
            atomicAdd(out.counts + 1, v);
            atomicAdd(out.counts + 2, t);
        }
        return;
    }
    if (MODE == 0) return;
    const double tau = (active && tri >= 0) ? round_trip_ns(R) : (double)INFINITY;
    // the staged records are dead: the same LDS now carries the waveform inputs
    wave_sync();
    float4* sub = reinterpret_cast<float4*>(wl);
    if (pair) {
        if (sc.shape == 0) pulse_pair<MAXCH, 0>(sc, pulses, out, first, sub, tau, P, tri, active);
        else pulse_pair<MAXCH, 1>(sc, pulses, out, first, sub, tau, P, tri, active);
    } else if (sc.shape == 0) {
        for (int q = 0; q < npw; ++q)
            pulse_phase<MAXCH, true, true, 0, CHUNK>(sc, pulses, out, first + q, q * S, sub, true, tau, P, tri);
    } else {
        for (int q = 0; q < npw; ++q)
            pulse_phase<MAXCH, true, true, 1, CHUNK>(sc, pulses, out, first + q, q * S, sub, true, tau, P, tri);
    }
}

template <int MAXCH, int MODE, bool CHUNK, bool VOX>
__device__ __forceinline__ void simulate_body(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                                              const OutDev& out, long long first, long long count, int ring_mask,
                                              int wl_bytes)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int waves = blockDim.x / kWave;
    unsigned char* wl = smem + (threadIdx.x / kWave) * wl_bytes;
    int* ring = reinterpret_cast<int*>(smem + wl_bytes * waves);
    long long wave = (long long)blockIdx.x * waves + threadIdx.x / kWave;
    long long p0 = wave * sc.P_w;
    if (p0 >= count) return;
    long long left = count - p0;
    int npw = left < sc.P_w ? (int)left : sc.P_w;
    process_wave<MAXCH, MODE, CHUNK, VOX>(scene, sc, pulses, out, first + p0, npw, ring, ring_mask, wl);
}

// Several pulses per wavefront: six wavefronts per SIMD (80 registers).
template <int MAXCH, int MODE, bool VOX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_simulate(SceneDev scene,
    ScannerDev sc, PulsesDev pulses, OutDev out, long long first, long long count, int ring_mask, int wl_bytes)
{
    simulate_body<MAXCH, MODE, false, VOX>(scene, sc, pulses, out, first, count, ring_mask, wl_bytes);
}

// One pulse per wavefront (candidate lists staged in chunks and culled): five
// wavefronts per SIMD, whose 96 registers hold the chunk loop without spills.
template <int MAXCH, int MODE, bool VOX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_simulate1(SceneDev scene,
    ScannerDev sc, PulsesDev pulses, OutDev out, long long first, long long count, int ring_mask, int wl_bytes)
{
    simulate_body<MAXCH, MODE, true, VOX>(scene, sc, pulses, out, first, count, ring_mask, wl_bytes);
}

// Waveform from stored subrays (KIND 0) or returns from stored waveforms (KIND 1).
template <int MAXCH, int KIND>
__global__ __launch_bounds__(256) void k_wave(ScannerDev sc, PulsesDev pulses, OutDev out, long long first,
                                              long long count)
{
    __shared__ float4 lds[4][kWave];
    float4* sub = lds[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int waves = blockDim.x / kWave;
    long long wave = (long long)blockIdx.x * waves + threadIdx.x / kWave;
    long long p0 = wave * sc.P_w;
    if (p0 >= count) return;
    long long left = count - p0;
    int npw = left < sc.P_w ? (int)left : sc.P_w;
    const int S = sc.S;
    const int pl = lane / S, k = lane - pl * S;
    bool attrib = KIND == 0 || (out.sub_tri && out.sub_range && out.sub_power);
    int tri = -1;
    double R = INFINITY;
    float P = 0.0f;
    if (attrib && pl < npw) {
        long long o = (first + p0 + pl) * out.sub_stride + k;
        tri = out.sub_tri[o];
        if (tri >= 0) {
            R = out.sub_range[o];
            P = out.sub_power[o];
        }
    }
    const double tau = tri >= 0 ? round_trip_ns(R) : (double)INFINITY;
    for (int q = 0; q < npw; ++q) {
        const long long p = first + p0 + q;
        if (KIND == 0) {
            if (sc.shape == 0) pulse_phase<MAXCH, true, false, 0>(sc, pulses, out, p, q * S, sub, true, tau, P, tri);
            else pulse_phase<MAXCH, true, false, 1>(sc, pulses, out, p, q * S, sub, true, tau, P, tri);
        } else {
            if (sc.shape == 0) pulse_phase<MAXCH, false, true, 0>(sc, pulses, out, p, q * S, sub, attrib, tau, P, tri);
            else pulse_phase<MAXCH, false, true, 1>(sc, pulses, out, p, q * S, sub, attrib, tau, P, tri);
        }
    }
}

// Batched, grouped by scanner: one launch per scanner of a batch over its
// segments' wave-tiles, one wavefront per tile.  The segment holding a tile is
// found by a wave-uniform binary search; the wavefront then runs exactly as in
// a launch of that segment alone (same kernel layout, same results).
template <int MAXCH, bool CHUNK, bool VOX>
__device__ __forceinline__ void grouped_body(const SceneDev& scene, const ScannerDev& sc, const GroupDev& g,
                                             const PulsesDev& pulses, const OutDev& out, int ring_mask, int wl_bytes)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int waves = blockDim.x / kWave;
    unsigned char* wl = smem + (threadIdx.x / kWave) * wl_bytes;
    int* ring = reinterpret_cast<int*>(smem + wl_bytes * waves);
    const long long tile = g.tile0 + (long long)blockIdx.x * waves + threadIdx.x / kWave;
    if (tile >= g.tile1) return;
    int lo = 0, hi = g.n_seg - 1;
    while (lo < hi) {  // last segment whose first tile <= tile
        const int mid = (lo + hi + 1) >> 1;
        if (g.tile_off[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    const long long p = g.pulse_off[lo] + (tile - g.tile_off[lo]) * sc.P_w;
    const long long left = g.pulse_end[lo] - p;
    const int npw = left < sc.P_w ? (int)left : sc.P_w;
    process_wave<MAXCH, 1, CHUNK, VOX>(scene, sc, pulses, out, p, npw, ring, ring_mask, wl);
}

template <int MAXCH, bool VOX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_grouped(SceneDev scene,
    ScannerDev sc, GroupDev g, PulsesDev pulses, OutDev out, int ring_mask, int wl_bytes)
{
    grouped_body<MAXCH, false, VOX>(scene, sc, g, pulses, out, ring_mask, wl_bytes);
}

template <int MAXCH, bool VOX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_grouped1(SceneDev scene,
    ScannerDev sc, GroupDev g, PulsesDev pulses, OutDev out, int ring_mask, int wl_bytes)
{
    grouped_body<MAXCH, true, VOX>(scene, sc, g, pulses, out, ring_mask, wl_bytes);
}

// Persistent batched kernel: wavefronts take chunks of wave-tiles from a global counter.
template <int MAXCH, bool VOX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_persistent(SceneDev scene, BatchDev batch, PulsesDev pulses,
                                                    OutDev out, int ring_mask, int wl_bytes)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int waves = blockDim.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned char* wl = smem + (threadIdx.x / kWave) * wl_bytes;
    int* ring = reinterpret_cast<int*>(smem + wl_bytes * waves);
    // Each wavefront takes `chunk` consecutive wave-tiles per counter update, so
    // the single counter sees about n_tiles / chunk atomics instead of one per tile.
    const long long chunk = batch.chunk;
    while (true) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(batch.counter, (unsigned long long)chunk);
        // broadcast lane 0's value as a wave-uniform (scalar) value
        const unsigned t_lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)t);
        const unsigned t_hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(t >> 32));
        const long long first = (long long)(((unsigned long long)t_hi << 32) | t_lo);
        if (first >= batch.n_tiles) break;
        const long long last = first + chunk < batch.n_tiles ? first + chunk : batch.n_tiles;
        int lo = 0, hi = batch.n_seg - 1;
        while (lo < hi) {  // last segment whose first tile <= first
            int mid = (lo + hi + 1) >> 1;
            if (batch.tile_off[mid] <= first) lo = mid;
            else hi = mid - 1;
        }
        for (long long tile = first; tile < last; ++tile) {
            while (lo + 1 < batch.n_seg && batch.tile_off[lo + 1] <= tile) ++lo;
            const ScannerDev sc = batch.scanners[batch.seg_scanner[lo]];
            long long p = batch.pulse_off[lo] + (tile - batch.tile_off[lo]) * sc.P_w;
            long long left = batch.pulse_end[lo] - p;
            int npw = left < sc.P_w ? (int)left : sc.P_w;
            process_wave<MAXCH, 1, false, VOX>(scene, sc, pulses, out, p, npw, ring, ring_mask, wl);
            wave_sync();
        }
    }
}

// Pulses with more candidates than a list holds: one wavefront per pulse walks
// the tree with all of the pulse's subrays as a packet and writes each subray's
// closest leaf (or -1) into the pulse's candidate row, with the count word
// kWalked; the fused kernel then tests that one leaf per subray.
// `list` holds the pulses (indices from `first`) and ctr[0] their number, both
// written by the cone pass; past one pulse per wavefront of the grid, the
// wavefronts take pulses from ctr[1] until the list is done.  Scanners: sc0, or per segment of `batch` when batch.n_seg > 0.
// The stack holds kPacketCap entries: three per four-wide level, which the
// scene check bounds the same way as the cone pass's stack.
__global__ __launch_bounds__(256) void k_packets(SceneDev scene, ScannerDev sc0, BatchDev batch, PulsesDev pulses,
                                                 int* __restrict__ cand, const int* __restrict__ list,
                                                 unsigned long long* ctr, long long first)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    int* stack = reinterpret_cast<int*>(smem);  // kPacketCap entries per wavefront, interleaved
    const unsigned long long n = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the first pulse of each wavefront is its index in the grid; later ones come
    // from the counter, so wavefronts without work never touch it
    const unsigned long long n_waves = (unsigned long long)gridDim.x * (blockDim.x / kWave);
    unsigned long long i = (unsigned long long)blockIdx.x * (blockDim.x / kWave) +
                           (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    int visits = 0, tests = 0;
    while (i < n) {
        const long long p = first + list[i];
        const ScannerDev* scp = &sc0;
        if (batch.n_seg > 0) {
            int lo = 0, hi = batch.n_seg - 1;
            while (lo < hi) {  // last segment whose first pulse <= p
                const int mid = (lo + hi + 1) >> 1;
                if (batch.pulse_off[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            scp = batch.scanners + batch.seg_scanner[lo];
        }
        const int S = scp->S;
        Ray r;
        const bool on = lane < S && setup_ray(pulses.origins + 3 * p, pulses.dirs + 3 * p, scp->pattern + 5 * lane, r);
        Hit h;
        h.t = INFINITY;
        h.leaf = -1;
        h.orig = 0x7fffffff;
        if (__ballot(on)) packet_walk<false>(scene, r, on, h, stack, kPacketCap, visits, tests);
        int* row = cand + p * (kCandMax + 1);
        if (lane < S) row[1 + lane] = h.leaf;
        if (lane == 0) row[0] = kWalked;
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(ctr + 1, 1ull);
        const unsigned t_lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)t);
        const unsigned t_hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(t >> 32));
        i = n_waves + (((unsigned long long)t_hi << 32) | t_lo);
    }
}

inline size_t sim_lds_bytes(int block, int ring, int wl_bytes)
{
    return (size_t)wl_bytes * (block / kWave) + sizeof(int) * (size_t)ring * block;
}

// ------------------------------------------------------------------ two-level scenes
//
// Scene parts kept once and placed by instances (Sec. 3.5: a part loaded several
// times with transforms; Sec. 5.1).  A pulse's subrays walk, as one packet, the
// top-level tree of the instances' boxes; in each instance reached they walk the
// part's tree with the ray mapped into the part's frame (O' = A^-1 (O - t), D' = A^-1 D, so the
// ray parameter, and with it every distance and the culling, is the world one),
// and tests each leaf's triangle as placed: vertices ((A_i0 x + A_i1 y) + A_i2 z)
// + t_i in FP64 rounded once to FP32, then the world-frame watertight test.
// These are exactly the triangles and the test of the expanded scene, so hits,
// distances and powers are the same bit for bit; the device holds the parts
// once.  Box tests in the part's frame are padded by the instance's pad_local,
// which covers the rounding of the placed vertices mapped back through A^-1.

// Placed vertex of an instance (the arithmetic of k_instance_verts).
__device__ __forceinline__ void place(const InstDev& I, float4 v, const Ray& r, double* w)
{
#pragma clang fp contract(off)
    const double x = v.x, y = v.y, z = v.z;
    for (int i = 0; i < 3; ++i) {
        const double* a = I.m + 4 * i;
        double q = a[0] * x;
        q = q + a[1] * y;
        q = q + a[2] * z;
        q = q + a[3];
        w[i] = (double)(float)q - r.O[i];
    }
}

// Box constants of the ray mapped into an instance's part frame.
__device__ __forceinline__ void local_box(const InstDev& I, const PartDev& P, const Ray& r, RayBox& b)
{
#pragma clang fp contract(off)
    double o[3], d[3];
    for (int i = 0; i < 3; ++i) {
        const double* a = I.inv + 4 * i;
        o[i] = ((a[0] * r.O[0] + a[1] * r.O[1]) + a[2] * r.O[2]) + a[3];
        d[i] = (a[0] * r.D[0] + a[1] * r.D[1]) + a[2] * r.D[2];
    }
    const double omax = fmax(fmax(fabs(o[0]), fabs(o[1])), fabs(o[2]));
    const double pad = (omax + (double)P.mag + 1.0) * 1.9073486328125e-06 + (double)I.pad_local;
    for (int i = 0; i < 3; ++i) {
        float di = (float)d[i];
        if (fabsf(di) < 1e-30f) di = copysignf(1e-30f, di);
        const float inv = 1.0f / di;
        b.inv[i] = inv;
        b.oim[i] = (float)(o[i] + pad) * inv;
        b.oip[i] = (float)(o[i] - pad) * inv;
    }
}

struct Hit2 {
    double t;
    int id;     // scene triangle id (instance's first id + the part's index)
    int inst;
    int leaf;   // the part's leaf
};

constexpr int kTopStack = 48;    // top-level depth limit (checked on the host)

__device__ __forceinline__ void leaf_test2(const InstDev& I, const PartDev& P, int j, int li, const Ray& r, Hit2& h,
                                           float& tcull)
{
    const float4 V0 = P.tris[3 * li], V1 = P.tris[3 * li + 1], V2 = P.tris[3 * li + 2];
    double a[3], b[3], c[3];
    place(I, V0, r, a);
    place(I, V1, r, b);
    place(I, V2, r, c);
    const double t = r.kz == 2 ? woop_t<2>(r, a, b, c, h.t)
                               : (r.kz == 1 ? woop_t<1>(r, a, b, c, h.t) : woop_t<0>(r, a, b, c, h.t));
    const int id = I.tri_base + __float_as_int(V0.w);
    if (!(t > 0.0 && (t < h.t || (t == h.t && id < h.id)))) return;
    h.t = t;
    h.id = id;
    h.inst = j;
    h.leaf = li;
    float tf = (float)t;
    if ((double)tf < t) tf = nextafterf(tf, INFINITY);
    tcull = tf;
}

// One part walked by the wavefront as a packet (as packet_walk does for a
// scene): the four-wide records, each lane's ray in the part's frame and its
// own culling distance, a child entered when any lane's box test passes,
// nearest first by the first lane's entry distance; a uniform stack of `cap`
// entries at st (3 per four-wide level; the host bounds the part's depth).
__device__ __forceinline__ void part_packet(const InstDev& I, const PartDev& P, int j, const Ray& r, bool on,
                                            int leader, Hit2& h, float& tcull, int* __restrict__ st, int cap)
{
    const int lane = threadIdx.x & (kWave - 1);
    if (P.n_tri <= 0) return;
    RayBox lb;
    local_box(I, P, r, lb);
    const int n_int = P.n_tri - 1;
    int node = P.root;
    int sp = 0;
    for (int guard = 2 * P.n_tri + 64; guard > 0; --guard) {
        if (node >= 0) {
            if (node >= n_int) break;  // only a corrupted structure gets here
            const float4* nd = P.nodes4 + 8 * node;
            const float4 LX = nd[0], LY = nd[1], LZ = nd[2], HX = nd[3], HY = nd[4], HZ = nd[5], RF = nd[6];
            int rf[4] = {__float_as_int(RF.x), __float_as_int(RF.y), __float_as_int(RF.z), __float_as_int(RF.w)};
            float t[4];
            bool hit[4];
            hit[0] = on && rf[0] != kEmpty4 && box_hit(lb, LX.x, LY.x, LZ.x, HX.x, HY.x, HZ.x, tcull, t[0]);
            hit[1] = on && rf[1] != kEmpty4 && box_hit(lb, LX.y, LY.y, LZ.y, HX.y, HY.y, HZ.y, tcull, t[1]);
            hit[2] = on && rf[2] != kEmpty4 && box_hit(lb, LX.z, LY.z, LZ.z, HX.z, HY.z, HZ.z, tcull, t[2]);
            hit[3] = on && rf[3] != kEmpty4 && box_hit(lb, LX.w, LY.w, LZ.w, HX.w, HY.w, HZ.w, tcull, t[3]);
            float key[4];
            for (int i = 0; i < 4; ++i) {
                const float lt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hit[i] ? t[i] : 3e38f), leader));
                key[i] = __ballot(hit[i]) ? lt : INFINITY;
            }
#define VLS_CX(a, b)                                            \
    if (key[b] < key[a]) {                                      \
        const float kt = key[a]; key[a] = key[b]; key[b] = kt; \
        const int rr = rf[a]; rf[a] = rf[b]; rf[b] = rr;       \
    }
            VLS_CX(0, 1) VLS_CX(2, 3) VLS_CX(0, 2) VLS_CX(1, 3) VLS_CX(1, 2)
#undef VLS_CX
            for (int q = 3; q >= 1; --q) {
                if (key[q] < INFINITY && sp < cap) {
                    if (lane == 0) st[sp] = rf[q];
                    ++sp;
                }
            }
            if (key[0] < INFINITY) {
                node = rf[0];
                continue;
            }
        } else {
            if (~node >= P.n_tri) break;  // only a corrupted structure gets here
            if (on) leaf_test2(I, P, j, ~node, r, h, tcull);
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(st[sp]);
    }
}

// The subrays of one pulse (lanes with `on`) through a two-level scene: the
// top-level binary tree walked as a packet (a child entered when any lane's
// box test passes, nearer first by the first lane), and each instance reached
// walked by part_packet.  top / low: the wavefront's uniform stacks.
__device__ __forceinline__ Hit2 packet_walk2(const TwoLevelDev& tl, const Ray& r, bool on, int* __restrict__ top,
                                             int* __restrict__ low)
{
    const int lane = threadIdx.x & (kWave - 1);
    Hit2 h;
    h.t = INFINITY;
    h.id = 0x7fffffff;
    h.inst = -1;
    h.leaf = -1;
    const unsigned long long onm = __ballot(on);
    if (tl.n_leaves <= 0 || !onm) return h;
    const int leader = __ffsll((long long)onm) - 1;
    RayBox rb;
    setup_box(r, tl.mag, rb);
    float tcull = INFINITY;
    int sp = 0;
    int node = tl.root;
    const int n_int = tl.n_leaves - 1;
    for (int budget = 2 * tl.n_leaves + 64; budget > 0; --budget) {
        if (node >= n_int || ~node >= tl.n_leaves) break;
        if (node >= 0) {
            const float4* nd = tl.nodes + 4 * node;
            const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
            float tl_ = 0.0f, tr_ = 0.0f;
            const bool hl = on && box_hit(rb, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tcull, tl_);
            const bool hr = on && box_hit(rb, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tcull, tr_);
            const int cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
            const float kl = __ballot(hl) ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hl ? tl_ : 3e38f), leader)) : INFINITY;
            const float kr = __ballot(hr) ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hr ? tr_ : 3e38f), leader)) : INFINITY;
            if (kl < INFINITY && kr < INFINITY) {
                if (sp < kTopStack) {
                    if (lane == 0) top[sp] = kl <= kr ? cr : cl;
                    ++sp;
                }
                node = kl <= kr ? cl : cr;
                continue;
            }
            if (kl < INFINITY) { node = cl; continue; }
            if (kr < INFINITY) { node = cr; continue; }
        } else {
            const int j = __float_as_int(tl.tris[3 * (~node)].w);
            if (j >= 0 && j < tl.n_inst) {
                const InstDev& I = tl.inst[j];
                part_packet(I, tl.parts[I.part], j, r, on, leader, h, tcull, low, kPacketCap);
            }
        }
        if (sp == 0) break;
        --sp;
        node = __builtin_amdgcn_readfirstlane(top[sp]);
    }
    return h;
}

// One wavefront per pulse, one lane per subray.
__global__ __launch_bounds__(256) void k_trace2(TwoLevelDev tl, ScannerDev sc, PulsesDev pulses, OutDev out,
                                                long long first, long long count)
{
    __shared__ int stacks[4][kTopStack + kPacketCap];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const long long q = (long long)blockIdx.x * (blockDim.x / kWave) + w;
    if (q >= count) return;
    const int S = sc.S;
    const int k = lane;
    const long long p = first + q;
    Ray r;
    const bool on = k < S && setup_ray(pulses.origins + 3 * p, pulses.dirs + 3 * p, sc.pattern + 5 * k, r);
    const Hit2 h = packet_walk2(tl, r, on, stacks[w], stacks[w] + kTopStack);
    if (k >= S) return;
    int tri = -1;
    double R = INFINITY;
    float cs = 0.0f, P = 0.0f;
    if (on && h.inst >= 0) {
        const InstDev& I = tl.inst[h.inst];
        const PartDev& Pt = tl.parts[I.part];
        const float4 V0 = Pt.tris[3 * h.leaf], V1 = Pt.tris[3 * h.leaf + 1], V2 = Pt.tris[3 * h.leaf + 2];
        double a[3], b[3], c[3];
        place(I, V0, r, a);
        place(I, V1, r, b);
        place(I, V2, r, c);
        SceneDev none{};
        shade(r, a, b, c, h.t, (float)(sc.power_c * sc.pattern[5 * k + 4]), Pt.refl[__float_as_int(V0.w)], none, 0,
              cs, P);
        tri = h.id;
        R = h.t;
    }
    const long long o = p * out.sub_stride + k;
    if (out.sub_tri) out.sub_tri[o] = tri;
    if (out.sub_range) out.sub_range[o] = R;
    if (out.sub_cos) out.sub_cos[o] = cs;
    if (out.sub_power) out.sub_power[o] = P;
}

}  // namespace

hipError_t launch_simulate(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                           long long first, long long count, int mode, const LaunchCfg& cfg, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const int block = cfg.block_waves * kWave;
    long long waves = (count + sc.P_w - 1) / sc.P_w;
    unsigned grid = (unsigned)((waves + cfg.block_waves - 1) / cfg.block_waves);
    const int wl = wave_lds_bytes(pulses.cand ? sc.P_w * staged_per_pulse(sc.P_w) : 0);
    size_t lds = sim_lds_bytes(block, cfg.stack_lds, wl);
    int mask = cfg.stack_lds - 1;
    // separate instantiations for scenes with voxels keep the others' code unchanged
    const bool vox = scene.vox.n_vox > 0;
#define VLS_SIM_LAUNCH_V(CH, MODE, VOX)                                                                       \
    do {                                                                                                     \
        if (sc.P_w == 1 && MODE != 2)                                                                        \
            hipLaunchKernelGGL((k_simulate1<CH, MODE, VOX>), dim3(grid), dim3(block), lds, stream, scene, sc, \
                               pulses, out, first, count, mask, wl);                                         \
        else                                                                                                 \
            hipLaunchKernelGGL((k_simulate<CH, MODE, VOX>), dim3(grid), dim3(block), lds, stream, scene, sc, \
                               pulses, out, first, count, mask, wl);                                         \
    } while (0)
#define VLS_SIM_LAUNCH(CH, MODE)               \
    do {                                       \
        if (vox) VLS_SIM_LAUNCH_V(CH, MODE, true);  \
        else VLS_SIM_LAUNCH_V(CH, MODE, false);     \
    } while (0)
    if (mode == 0) VLS_SIM_LAUNCH(4, 0);
    else if (mode == 2) VLS_SIM_LAUNCH(4, 2);
    else if (sc.n_bins <= 256) VLS_SIM_LAUNCH(4, 1);
    else if (sc.n_bins <= 512) VLS_SIM_LAUNCH(8, 1);
    else VLS_SIM_LAUNCH(16, 1);
#undef VLS_SIM_LAUNCH
#undef VLS_SIM_LAUNCH_V
    return hipGetLastError();
}

hipError_t launch_packets(const SceneDev& scene, const ScannerDev& sc0, const BatchDev& batch, const PulsesDev& pulses,
                          int* cand, const int* ovf_list, unsigned long long* ovf_ctr, long long first,
                          hipStream_t stream)
{
    if (scene.n_tri <= 0) return hipSuccess;
    // a fixed grid: the wavefronts find the number of pulses to walk on the device
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    // eight wavefronts per SIMD: the walks wait on dependent node fetches, and
    // more resident walks hide more of that latency (measured: 4 per SIMD is
    // 11 % slower on a vegetation scene, 16 per SIMD 5 % slower)
    const int block = 4 * kWave;
    const unsigned grid = (unsigned)(cus > 0 ? 8 * cus : 2048);
    const size_t lds = sizeof(int) * (size_t)kPacketCap * block / kWave;
    hipLaunchKernelGGL(k_packets, dim3(grid), dim3(block), lds, stream, scene, sc0, batch, pulses, cand, ovf_list,
                       ovf_ctr, first);
    return hipGetLastError();
}

hipError_t launch_waveform(const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out, long long first,
                           long long count, int mode, const LaunchCfg& cfg, hipStream_t stream)
{
    (void)cfg;
    if (count <= 0) return hipSuccess;
    const int block = 4 * kWave;
    long long waves = (count + sc.P_w - 1) / sc.P_w;
    unsigned grid = (unsigned)((waves + 3) / 4);
#define VLS_WAVE_LAUNCH(CH)                                                                                  \
    do {                                                                                                     \
        if (mode == 0)                                                                                       \
            hipLaunchKernelGGL((k_wave<CH, 0>), dim3(grid), dim3(block), 0, stream, sc, pulses, out, first, count); \
        else                                                                                                 \
            hipLaunchKernelGGL((k_wave<CH, 1>), dim3(grid), dim3(block), 0, stream, sc, pulses, out, first, count); \
    } while (0)
    if (sc.n_bins <= 256) VLS_WAVE_LAUNCH(4);
    else if (sc.n_bins <= 512) VLS_WAVE_LAUNCH(8);
    else VLS_WAVE_LAUNCH(16);
#undef VLS_WAVE_LAUNCH
    return hipGetLastError();
}

hipError_t launch_grouped(const SceneDev& scene, const ScannerDev& sc, const GroupDev& g, const PulsesDev& pulses,
                          const OutDev& out, const LaunchCfg& cfg, hipStream_t stream)
{
    const long long tiles = g.tile1 - g.tile0;
    if (tiles <= 0 || g.n_seg <= 0) return hipSuccess;
    const int block = cfg.block_waves * kWave;
    const unsigned grid = (unsigned)((tiles + cfg.block_waves - 1) / cfg.block_waves);
    const int wl = wave_lds_bytes(pulses.cand ? sc.P_w * staged_per_pulse(sc.P_w) : 0);
    const size_t lds = sim_lds_bytes(block, cfg.stack_lds, wl);
    const int mask = cfg.stack_lds - 1;
    const bool vox = scene.vox.n_vox > 0;
#define VLS_GROUPED_V(CH, VOX)                                                                                     \
    do {                                                                                                          \
        if (sc.P_w == 1)                                                                                          \
            hipLaunchKernelGGL((k_grouped1<CH, VOX>), dim3(grid), dim3(block), lds, stream, scene, sc, g, pulses, out, \
                               mask, wl);                                                                         \
        else                                                                                                      \
            hipLaunchKernelGGL((k_grouped<CH, VOX>), dim3(grid), dim3(block), lds, stream, scene, sc, g, pulses, out,  \
                               mask, wl);                                                                         \
    } while (0)
#define VLS_GROUPED(CH)                   \
    do {                                  \
        if (vox) VLS_GROUPED_V(CH, true); \
        else VLS_GROUPED_V(CH, false);    \
    } while (0)
    if (sc.n_bins <= 256) VLS_GROUPED(4);
    else if (sc.n_bins <= 512) VLS_GROUPED(8);
    else VLS_GROUPED(16);
#undef VLS_GROUPED
#undef VLS_GROUPED_V
    return hipGetLastError();
}

hipError_t launch_persistent(const SceneDev& scene, const BatchDev& batch, int max_bins, int staged_slots,
                             const PulsesDev& pulses, const OutDev& out, const LaunchCfg& cfg, int blocks,
                             hipStream_t stream)
{
    const int block = cfg.block_waves * kWave;
    const int wl = wave_lds_bytes(pulses.cand ? staged_slots : 0);
    size_t lds = sim_lds_bytes(block, cfg.stack_lds, wl);
    int mask = cfg.stack_lds - 1;
    hipError_t e = launch_fill_u64(batch.counter, 1, 0ull, stream);
    if (e != hipSuccess) return e;
    BatchDev b = batch;
    long long waves = (long long)blocks * cfg.block_waves;
    long long ch = batch.n_tiles / (waves * 16 > 0 ? waves * 16 : 1);
    b.chunk = (int)(ch < 1 ? 1 : (ch > 4096 ? 4096 : ch));
#define VLS_PERSISTENT(CH, VOX)                                                                                \
    hipLaunchKernelGGL((k_persistent<CH, VOX>), dim3(blocks), dim3(block), lds, stream, scene, b, pulses, out, mask, wl)
    const bool vox = scene.vox.n_vox > 0;
    if (max_bins <= 256) {
        if (vox) VLS_PERSISTENT(4, true);
        else VLS_PERSISTENT(4, false);
    } else if (max_bins <= 512) {
        if (vox) VLS_PERSISTENT(8, true);
        else VLS_PERSISTENT(8, false);
    } else {
        if (vox) VLS_PERSISTENT(16, true);
        else VLS_PERSISTENT(16, false);
    }
#undef VLS_PERSISTENT
    return hipGetLastError();
}

int persistent_occupancy_blocks(int max_bins, int staged_slots, bool vox, const LaunchCfg& cfg)
{
    const int block = cfg.block_waves * kWave;
    size_t lds = sim_lds_bytes(block, cfg.stack_lds, wave_lds_bytes(cfg.cone ? staged_slots : 0));
    int per_cu = 0;
    hipError_t e;
    if (max_bins <= 256)
        e = vox ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<4, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<4, false>, block, lds);
    else if (max_bins <= 512)
        e = vox ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<8, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<8, false>, block, lds);
    else
        e = vox ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<16, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<16, false>, block, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 1;
    return per_cu * cus;
}

hipError_t launch_trace2(const TwoLevelDev& tl, const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                         long long first, long long count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace2, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, stream, tl, sc, pulses, out, first,
                       count);
    return hipGetLastError();
}

}  // namespace vls
