// Internal types shared by the library's HIP translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace vls {

constexpr double kCmPerNs = 0.299792458;  // speed of light in m/ns (Sec. 3.4)
constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kMaxSpill = 112;            // traversal-stack entries per lane beyond the LDS ring
constexpr int kMaxRing = 32;
constexpr int kCandMax = 255;            // candidate leaves kept per pulse by the cone pass
static_assert(kCandMax >= kWave, "a packet walk writes one leaf per subray into the row");
constexpr int kEmpty4 = 0x7fffffff;       // unused slot of a four-wide record
constexpr int kConeRing = 16;            // LDS stack entries per lane of the cone pass
constexpr int kConeRingCover = 8;        // the same with cover tests (walks culled behind a cover stay shallow)
constexpr int kWalked = -2;              // count word kWalked: the row holds one leaf per subray
constexpr int kPacketCap = 128;          // stack entries of a packet walk (3 per four-wide level)

// Cone-pass workspace for n pulses: candidate rows [n][kCandMax + 1], then the
// list of pulses that overflowed [n], then two counters (overflow count, work),
// then each pulse's basis [n][5] doubles (see dev::Basis).
constexpr size_t cone_ws_ints(long long n) { return (size_t)(kCandMax + 1) * n + n + (n & 1) + 4 + 10 * (size_t)n; }
inline int* cone_ws_list(int* ws, long long n) { return ws + (size_t)(kCandMax + 1) * n; }
inline unsigned long long* cone_ws_ctr(int* ws, long long n)
{
    return reinterpret_cast<unsigned long long*>(ws + (size_t)(kCandMax + 1) * n + n + (n & 1));
}
inline double* cone_ws_basis(int* ws, long long n)
{
    return reinterpret_cast<double*>(ws + (size_t)(kCandMax + 1) * n + n + (n & 1) + 4);
}
// Long candidate lists: a pulse that overflows its row is walked again by a
// second cone pass with room for kLongMax candidates, in one of at most
// kLongPulses rows of a separate workspace (4 KiB each); its row then holds the count (past
// kCandMax) and the long row's index.  Long-list workspace for n pulses: the
// rows [min(n, kLongPulses)][kLongMax], then the list of pulses left for the
// packet walk [n], then two 64-bit counters (long-list count, packet-list count).
constexpr int kLongMax = 1024;
constexpr long long kLongPulses = 262144;
// With long lists at hand the first pass stops a pulse's walk at kCandFirst
// candidates: the long walkers then run together in the second pass instead of
// holding up the wavefronts of the first (measured on the vegetation workload:
// 19.2 ms per step against 21.0 ms at 255, 20.1 at 127, 20.3 at 191 and 223).
constexpr int kCandFirst = 159;
__host__ __device__ constexpr long long long_rows(long long n) { return n < kLongPulses ? n : kLongPulses; }
constexpr size_t long_ws_ints(long long n) { return (size_t)kLongMax * long_rows(n) + n + (n & 1) + 4; }
inline int* long_ws_list(int* w, long long n) { return w + (size_t)kLongMax * long_rows(n); }
inline unsigned long long* long_ws_ctr(int* w, long long n)
{
    return reinterpret_cast<unsigned long long*>(w + (size_t)kLongMax * long_rows(n) + n + (n & 1));
}
// The allocation-free simulate entry point keeps its workspace in a fixed device
// array: the subray table of its one scanner (5 doubles per subray), then the
// cone-pass workspace above for at most kNoAllocMaxPulses pulses.
constexpr long long kNoAllocMaxPulses = 32768;
constexpr size_t kNoAllocPatternBytes = 5 * kWave * sizeof(double);
constexpr size_t kNoAllocScratchBytes = kNoAllocPatternBytes + sizeof(int) * cone_ws_ints(kNoAllocMaxPulses);
static_assert(kNoAllocPatternBytes % 256 == 0, "the candidate workspace starts 256-byte aligned");
constexpr int kMaxLevel = 4096;          // depth cap of the build's level lists
constexpr int kCandStaged = 16;          // of which the first ones are staged in LDS by the fused kernel
// Candidates staged per pulse: one per lane of the wavefront, so 64 for one pulse
// per wavefront, 16 for two to four (0 beyond: nothing staged).  The fused kernel
// relies on both being powers of two.
__host__ __device__ constexpr int staged_per_pulse(int pulses_per_wave)
{
    return pulses_per_wave == 1 ? kWave : (pulses_per_wave <= 4 ? kCandStaged : 0);
}

// One scanner as the kernels see it (everything derived on the host in FP64).
struct ScannerDev {
    const double* pattern;  // [S][5]: cos a, sin a, cos phi, sin phi, weight
    int S;                  // subrays per pulse
    int P_w;                // pulses per wavefront = 64 / S
    int n_bins;
    int K;
    int shape;              // 0 Gaussian, 1 Eq. 3
    float bin_ns;
    double bin_d;           // bin width in FP64 (bin times t0 + j bin)
    float neg_k;            // Gaussian: -log2(e) / (2 sigma^2); Eq. 3: -log2(e)
    float inv_tau;          // Eq. 3: 1 / tau
    float cut_lo;           // a subray contributes to bins with s in [-cut_lo, cut_hi] ns
    float cut_hi;
    float inv_bin;          // 1 / bin_ns
    double t_pre;           // window starts t_pre before the first echo
    double s_peak;          // peak offset of the pulse shape (0 Gaussian, 2 tau Eq. 3)
    double power_c;         // peak * eff * D^2 / 4
    double thr_abs;
    double thr_rel;
    double tan_max;         // tan of the largest subray angle (outer ring)
    double range_noise;     // ranging error's standard deviation (m), 0: none
    unsigned long long noise_seed;
    double vox_c;           // voxel echoes (Eq. 7): power_c / (pi beta^2), beta the full divergence
};

// A transmissive voxel grid (see voxels.h); n_vox == 0: none.
struct VoxDev {
    const float* pad;       // [nz][ny][nx] plant area density
    const double* lut;      // [n_lut][2]: vertical component (strictly increasing), g
    double origin[3];
    double size;            // voxel side
    int nx, ny, nz, n_lut;
    unsigned long long seed;
    long long n_vox;        // nx * ny * nz
};

// Binary LBVH: node = 4 x float4 (64 B): left box lo.xyz hi.x | hi.yz, right lo.xy |
// right lo.z hi.xyz | refs (left, right, parent, 0) as int bits.  A ref >= 0 is an
// internal node; ref < 0 is leaf ~ref.  Leaf record = 3 x float4 (48 B):
// v0.xyz + original triangle index (int bits) | v1.xyz + 0 | v2.xyz + 0.
struct SceneDev {
    const float4* nodes;
    const float4* nodes4;   // [n_tri-1][8]: four-wide records (grandchildren of each node)
    const float4* tris;
    const float* refl;      // by original triangle index
    const float* bounds;    // [13]: vertex lo.xyz hi.xyz, centroid lo.xyz hi.xyz, max |coordinate|
    const float* verts;     // [n_vert][3] current vertices (adjoint)
    const int32_t* tri_idx; // [n_tri][3] vertex indices (adjoint)
    int root;
    int n_tri;
    VoxDev vox;
    const float* spec_k;    // per-triangle specularity, or null (Lambertian)
    const float* spec_n;    // per-triangle Phong exponent
};

struct PulsesDev {
    const double* origins;
    const float* dirs;
    const double* t0_in;    // may be null
    long long n;
    const double* basis;    // [n][5] each pulse's basis from the cone pass (n, a, b), or null
    const int* cand;        // [n][kCandMax + 1] candidate leaves from the cone pass, or null:
                            // entry 0 = count (-1 = overflow, use full traversal; kWalked:
                            // one leaf per subray from a packet walk), then leaf ids; a
                            // count past kCandMax: entry 1 is a row of cand_long
    const int* cand_long;   // [rows][kLongMax] long candidate lists, or null
};

// The leaf ids of a pulse's candidate row (count nc > 0 read from row[0]).
__host__ __device__ inline const int* cand_ids(const int* row, int nc, const int* cand_long)
{
    return nc > kCandMax ? cand_long + (size_t)row[1] * kLongMax : row + 1;
}

struct OutDev {
    int32_t* sub_tri;
    double* sub_range;
    float* sub_cos;
    float* sub_power;
    int sub_stride;
    int pad_;
    float* wf;
    double* t0;
    int32_t* n_ret;
    float* ret_range;
    float* ret_amp;
    int32_t* ret_tri;
    int32_t* ret_bin;
    unsigned long long* counts;  // diagnostic: subrays, node visits, triangle tests (mode 2)
};

// Segmented batch for the persistent kernel.
struct BatchDev {
    const long long* tile_off;    // [n_seg+1] first wave-tile of each segment
    const long long* pulse_off;   // [n_seg] first pulse of each segment
    const long long* pulse_end;   // [n_seg]
    const int* seg_scanner;       // [n_seg]
    const ScannerDev* scanners;   // [n_scanners]
    unsigned long long* counter;  // work counter (reset before each launch)
    int n_seg;
    int chunk;                    // wave-tiles taken per counter update
    long long n_tiles;
};

// One scanner's segments of a batch, numbered in the batch's scanner-grouped
// tile order: a launch covers tiles [tile0, tile1), segment i starting at tile
// tile_off[i] with pulses [pulse_off[i], pulse_end[i]).
struct GroupDev {
    const long long* tile_off;
    const long long* pulse_off;
    const long long* pulse_end;
    int n_seg = 0;
    long long tile0 = 0, tile1 = 0;
};

// Two-level scenes (scene parts kept once, placed by instances; see trace.hip
// k_trace2).  A part: its own LBVH over its triangles in its own frame.
struct PartDev {
    const float4* nodes;
    const float4* nodes4;   // four-wide records
    const float4* tris;     // leaf records; .w of the first row = the part's triangle index
    const float* refl;      // by the part's triangle index
    int root;
    int n_tri;
    float mag;              // largest |coordinate| of the part's vertices
    int pad_;
};

// An instance: x -> A x + t (m, rows [A_i0 A_i1 A_i2 t_i]) and its inverse
// (inv, the same layout), the part, the scene id of its first triangle, and the
// extra box padding in the part's frame that covers the FP32 rounding of the
// placed vertices.
struct InstDev {
    double m[12];
    double inv[12];
    int part;
    int tri_base;
    float pad_local;
    int pad_;
};

// The top level: an LBVH over the instances' boxes in the scene's frame (leaf
// records hold each box as the degenerate triangle (lo, hi, lo); .w = the
// instance index).
struct TwoLevelDev {
    const float4* nodes;
    const float4* tris;
    const InstDev* inst;
    const PartDev* parts;
    int root;
    int n_leaves;
    int n_inst;
    float mag;
};

// A survey as the pulse generator sees it (see survey.hip).
struct SurveyDev {
    int n_wp;
    int deflector;   // 0 polygon, 1 swing, 2 conic, 3 fibre
    int n_fibres;
    int platform;    // 0 LinearPath: table rows (x, y, z, path length, cos yaw, sin yaw);
                     // 1 Multicopter: rows (x, y, z, leg start time, leg duration,
                     //   leg length, start yaw, end yaw);
                     // 2 Multicopter with smooth turns: one row of kSmoothRow per
                     //   piece of the path (see survey.hip), n_piece rows
    double speed, prf, freq, angle, t0, noise, accel;
    uint64_t seed;
    int n_piece;         // smooth turns: pieces of the path
    double path_len;     // smooth turns: length of the whole path
    double t_end;        // smooth turns: arrival at the last waypoint
};
// A piece of a smooth-turn path: path length at its start, its length, 1 for an
// arc (0 straight), radius, bank, start point (straight) or centre (arc),
// direction (straight) or tangent at the start (arc), unit vector toward the
// centre (arc), two unused.
constexpr int kSmoothRow = 16;

struct LaunchCfg {
    int block_waves = 1;
    int stack_lds = 16;
    int persistent_blocks = 0;
    int pack = 0;  // 0: floor(64/S) pulses per wavefront; 1: one pulse per wavefront
    int cone = 1;  // 1: one cone traversal per pulse collects candidate triangles for its subrays
    int cover_off = 0;  // 1: the cone traversal runs no cover tests
    int grouped = 1;    // batches: 1 one launch per scanner over its segments' tiles, 0 the persistent kernel
};

// ---- host-side launchers (defined in the .hip files) ----
// All return hipSuccess or the first HIP error; kernels are enqueued on `stream`.

struct BvhBuffers {
    float4* nodes = nullptr;      // [max(n_tri-1,1)][4]
    float4* nodes4 = nullptr;     // [max(n_tri-1,1)][8] four-wide records, rebuilt with every refit
    float4* tris = nullptr;       // [n_tri][3]
    float* refl = nullptr;        // [n_tri]
    float* verts = nullptr;       // [n_vert][3]
    int32_t* tri_idx = nullptr;   // [n_tri][3]
    int32_t* leaf_parent = nullptr;   // [n_tri]
    int32_t* node_parent = nullptr;   // [n_tri-1]
    int32_t* leaf_tri = nullptr;      // [n_tri] original index per leaf
    unsigned long long* morton = nullptr;  // [n_tri] sorted keys
    int32_t* node_depth = nullptr;    // [n_tri-1] steps from the root
    int32_t* level_order = nullptr;   // [n_tri-1] internal nodes by depth, shallowest first
    std::vector<long long> level_off; // depth d occupies level_order[level_off[d], level_off[d + 1])
    float* bounds = nullptr;          // [32]: [0..12] as in SceneDev, [13] depth (uint bits), [16..28] scratch
    int64_t n_tri = 0, n_vert = 0;
};

// Device check of a copied mesh (indices in range, finite vertices): bad gets bit
// 0 for an index out of range, bit 1 for a non-finite coordinate.  Synchronises.
hipError_t mesh_check(const BvhBuffers& b, hipStream_t stream, unsigned& bad);
hipError_t bvh_build(BvhBuffers& b, hipStream_t stream, std::string& err);
// Stable LSD radix sort of (key, value) pairs by the low 8 * passes bits of the
// keys (passes even: the result ends in keys / vals; the second pair of arrays
// is the ping-pong buffer); hist holds radix_sort_hist_words(n) words.
long long radix_sort_hist_words(long long n);
hipError_t radix_sort_pairs(unsigned long long* keys, int32_t* vals, unsigned long long* keys2, int32_t* vals2,
                            unsigned* hist, long long n, int passes, hipStream_t stream);
hipError_t bvh_refit(BvhBuffers& b, hipStream_t stream);
hipError_t bvh_update_vertices(BvhBuffers& b, hipStream_t stream);

hipError_t launch_simulate(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                           const OutDev& out, long long first, long long count, int mode,
                           const LaunchCfg& cfg, hipStream_t stream);
hipError_t launch_waveform(const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                           long long first, long long count, int mode, const LaunchCfg& cfg, hipStream_t stream);
// staged_slots: the most candidate records any of the batch's scanners stages per
// wavefront (pulses per wavefront * staged_per_pulse): it sizes that LDS.
// One launch over one scanner's segments of a batch (the fused kernel of its
// layout, one wavefront per tile, the segment found by a binary search).
hipError_t launch_grouped(const SceneDev& scene, const ScannerDev& sc, const GroupDev& g, const PulsesDev& pulses,
                          const OutDev& out, const LaunchCfg& cfg, hipStream_t stream);
hipError_t launch_persistent(const SceneDev& scene, const BatchDev& batch, int max_bins, int staged_slots,
                             const PulsesDev& pulses, const OutDev& out, const LaunchCfg& cfg, int blocks,
                             hipStream_t stream);
hipError_t launch_backward(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                           const int32_t* sub_tri, int sub_stride, const float* grad_wf, float* grad_refl,
                           float* grad_z, long long n_vert, const LaunchCfg& cfg, hipStream_t stream);
// The adjoint with sums in a fixed order (per-entry contributions, a stable sort
// by parameter, sums of each run in entry order): bitwise repeatable.  ws holds
// backward_det_bytes(n_pulses, S) bytes.
size_t backward_det_bytes(long long n_pulses, int S);
hipError_t launch_backward_det(const SceneDev& scene, const ScannerDev& sc, const PulsesDev& pulses,
                               const int32_t* sub_tri, int sub_stride, const float* grad_wf, float* grad_refl,
                               float* grad_z, long long n_vert, const LaunchCfg& cfg, void* ws, hipStream_t stream);
// Cone pass: pulses [first, first + count), cone slope tan_max (largest over the
// scanners in use).  Writes cand[p * (kCandMax + 1) ...]; counts (optional)
// accumulates node visits into counts[1].
// ovf_list / ovf_ctr (optional): pulses whose list overflows are appended to
// ovf_list (indices from `first`) and counted in ovf_ctr[0]; both counters are
// reset first.
// basis_out (optional): each pulse's basis, [p][5] doubles.
hipError_t launch_cone(const SceneDev& scene, double tan_max, const PulsesDev& pulses, int* cand, long long first,
                       long long count, const LaunchCfg& cfg, unsigned long long* counts, int* ovf_list,
                       unsigned long long* ovf_ctr, double* basis_out, hipStream_t stream,
                       int cap = kCandMax, bool cover = true);
// Second cone pass over the pulses that overflowed their rows (list, ctr from
// launch_cone): each gets a long row while rows last (its candidate row then
// holds the count and the long row's index), else it goes to list2 / ctr2 for
// the packet walk, as do pulses whose long list overflows too.
hipError_t launch_cone_long(const SceneDev& scene, double tan_max, const PulsesDev& pulses, int* cand,
                            const int* list, const unsigned long long* ctr, long long n, int* longw,
                            const LaunchCfg& cfg, hipStream_t stream);
// Packet walks of the overflowed pulses (see k_packets); batch.n_seg == 0: every
// pulse uses sc0.
hipError_t launch_packets(const SceneDev& scene, const ScannerDev& sc0, const BatchDev& batch, const PulsesDev& pulses,
                          int* cand, const int* ovf_list, unsigned long long* ovf_ctr, long long first,
                          hipStream_t stream);
// Echo width of the kept returns of pulses [first, first + count) (see echo.hip):
// list / list_ctr: workspace of count * K ints and one 64-bit counter.
hipError_t launch_echo_width(const ScannerDev& sc, const float* wf, const int32_t* n_ret, const int32_t* ret_bin,
                             float s0_bins, long long first, long long count, int* list,
                             unsigned long long* list_ctr, float* width, hipStream_t stream);
// Per-subray closest hits, power and incidence in a two-level scene (pulses
// [first, first + count) of one scanner); writes the out.sub_* arrays that are set.
hipError_t launch_trace2(const TwoLevelDev& tl, const ScannerDev& sc, const PulsesDev& pulses, const OutDev& out,
                         long long first, long long count, hipStream_t stream);
// Ranging error on the kept returns of pulses [first, first + count) of one scanner
// (nothing when its range_noise is 0; see survey.hip).
hipError_t launch_range_noise(const ScannerDev& sc, const int32_t* n_ret, float* ret_range, long long first,
                              long long count, hipStream_t stream);
// Pulses [first, first + count) of a survey; tab: per-waypoint table (see survey.hip).
hipError_t launch_generate(const SurveyDev& sv, const double* tab, long long first, long long count,
                           double* origins, float* dirs, hipStream_t stream);
// Scene parts (see instance.hip): the k instances of one part, aff [k][12] rows
// (A_i0, A_i1, A_i2, t_i), voff / toff [k] each instance's first scene vertex and
// triangle; *bad gets bit 0 for a part's vertex index out of range.
hipError_t launch_instances(const float* v, const int32_t* t, const float* refl, long long nv, long long nt,
                            const double* aff, const long long* voff, const long long* toff, long long k,
                            float* out_v, int32_t* out_t, float* out_r, unsigned* bad, hipStream_t stream);
// Candidate lists hold leaf indices; rewrite them as original triangle indices.
hipError_t launch_leaf_to_orig(const int32_t* leaf_tri, int* cand, long long n_pulses, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, long long n, unsigned long long v, hipStream_t stream);
int persistent_occupancy_blocks(int max_bins, int staged_slots, bool vox, const LaunchCfg& cfg);
// The allocation-free entry point's device scratch (kNoAllocScratchBytes) on
// `device`: its address, looked up once per device (see noalloc.hip).
hipError_t noalloc_scratch(int device, void** ptr);
// Writes a subray table (n doubles, n <= 5 * kWave) to device memory dst with one
// small kernel; the table travels as the kernel's argument.
hipError_t launch_store_pattern(const double* table, int n, double* dst, hipStream_t stream);

}  // namespace vls
