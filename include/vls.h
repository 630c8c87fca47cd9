/*
 * vls.h - C ABI of the MI355X (gfx950) virtual-laser-scanning library.
 *
 * The library computes the data-parallel hot path of full-waveform virtual
 * laser scanning as described for HELIOS++ (Winiwarter et al., "Virtual laser
 * scanning with HELIOS++", arXiv 2101.09154):
 *   - each pulse's beam is split into subrays on concentric rings (Sec. 3.4,
 *     Fig. 6) weighted by the Gaussian beam profile (Sec. 3.4, Eq. 1);
 *   - every subray is cast separately and stops at its first hit (Sec. 3.4),
 *     found through an acceleration structure over the triangles (Sec. 5.1;
 *     here a linear BVH instead of the paper's kD-tree);
 *   - its return power follows the laser radar equation (Sec. 5.2, Eq. 7)
 *     with incidence angle and per-triangle reflectance (Sec. 5.1);
 *   - the returned waveform is the sum of the subrays' pulse shapes
 *     (Sec. 3.4, Eq. 3, or a Gaussian pulse) shifted by their two-way travel
 *     times, sampled in bins over a window of bounded length (Sec. 5.4);
 *   - local maxima of the waveform become discrete returns (Sec. 3.4).
 * Readings where the paper is silent are the library's documented
 * conventions; they are listed next to each entry point.
 *
 * Conventions for every function:
 *   - returns vls_status; VLS_OK == 0; nothing throws across the ABI;
 *   - invalid arguments are detected before anything is enqueued;
 *   - device work is enqueued on the caller's HIP stream (hipStream_t passed
 *     as void*, NULL = the null stream) and is asynchronous unless stated;
 *   - device faults surface at the next synchronising call, e.g. vls_synchronize;
 *   - the caller owns every array it passes; the library owns contexts,
 *     scenes and graphs, freed by their *_destroy call;
 *   - a context (and everything created from it) is not thread-safe: calls on
 *     it come from one host thread at a time;
 *   - a context may be used with several streams: each stream gets its own
 *     workspaces (candidate lists, counters, echo-width and adjoint scratch),
 *     grown when a call needs more by stream-ordered allocation on that stream
 *     (hipMallocAsync / hipFreeAsync), so calls on different streams share no
 *     scratch memory and growing one does not synchronise the device; a
 *     stream must outlive the calls made on it until they have completed;
 *   - calls documented as synchronous (scene creation, statistics, the first
 *     upload of a scanner's subray table or of a batch's segment table, which
 *     are shared read-only by every stream) wait for their own copies.
 */
#ifndef VLS_H
#define VLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VLS_OK = 0,
    VLS_ERR_INVALID_ARG = 1,   /* NULL where required, bad sizes or parameters         */
    VLS_ERR_OUT_OF_MEMORY = 2, /* a device or host allocation failed                    */
    VLS_ERR_DEVICE = 3,        /* a HIP runtime call or a kernel failed                  */
    VLS_ERR_NOT_BUILT = 4,     /* reserved                                               */
    VLS_ERR_UNSUPPORTED = 5,   /* valid request outside what the library handles         */
    VLS_ERR_INTERNAL = 6       /* a C++ exception or an invariant failure inside the lib */
} vls_status;

enum { VLS_MEM_HOST = 0, VLS_MEM_DEVICE = 1 };
enum { VLS_PULSE_GAUSSIAN = 0, VLS_PULSE_EQ3 = 1 };

/* Limits of this build. */
#define VLS_MAX_SUBRAYS 64      /* subrays per pulse (one wavefront)            */
#define VLS_MAX_BINS 1024       /* waveform bins per pulse                       */
#define VLS_MAX_RETURNS 16      /* returns kept per pulse                        */
#define VLS_MAX_SCANNERS 64     /* scanner descriptions per batched call         */
#define VLS_MAX_CANDIDATES 255  /* triangles the cone pass lists per pulse       */

const char* vls_status_string(vls_status s);
/* Detail of the last failure on the calling thread; valid until the next vls_* call there. */
const char* vls_last_error(void);
int32_t vls_version(void);

typedef struct vls_context_s* vls_context;
typedef struct vls_scene_s* vls_scene;
typedef struct vls_graph_s* vls_graph;

/* A context binds one HIP device and caches per-scanner subray tables and the
 * launch configuration.  vls_context_create makes `hip_device` current. */
vls_status vls_context_create(int32_t hip_device, vls_context* out);
vls_status vls_context_destroy(vls_context ctx);

/* ------------------------------------------------------------------ scenes */

/* Triangle mesh (Sec. 5.1: a scene is a set of primitives, each with a material;
 * here triangles with a reflectance in [0, 1]).
 *   vertices    [n_vertices][3] float32, metres
 *   triangles   [n_triangles][3] int32 vertex indices (checked on the device
 *               by vls_scene_create)
 *   reflectance [n_triangles] float32
 *   memory      where the three arrays live: VLS_MEM_HOST or VLS_MEM_DEVICE.
 * n_triangles may be 0 (every subray misses).
 * There is no per-triangle object id: returns carry the index of the triangle
 * they are attributed to (ret_tri, an index into `triangles`), so a caller that
 * groups triangles into objects looks the object up as object_id[ret_tri]. */
typedef struct {
    const float* vertices;
    const int32_t* triangles;
    const float* reflectance;
    int64_t n_vertices;
    int64_t n_triangles;
    int32_t memory;
    int32_t reserved;
} vls_mesh_desc;

typedef struct {
    int64_t n_vertices;
    int64_t n_triangles;
    int64_t n_internal_nodes;   /* n_triangles - 1 (binary LBVH, one triangle per leaf)   */
    int64_t device_bytes;       /* bytes of device memory the scene holds                 */
    int32_t max_depth;          /* deepest leaf (root = 0)                                */
    int32_t max_supported_depth;/* deepest tree the per-subray traversal stack holds (the
                                   LDS ring plus 112 scratch entries); tracing a deeper
                                   scene returns VLS_ERR_UNSUPPORTED, and so does a scene
                                   deeper than 84 with the cone pass on                    */
    float bounds_lo[3];         /* vertex bounds                                          */
    float bounds_hi[3];
    float box_pad;              /* 0: node boxes are exact; traversal pads them per ray    */
    float reserved;
} vls_scene_stats;

/* Copies the mesh to the device and builds the acceleration structure: Morton
 * codes of triangle centroids (63 bits), radix sort, Karras (2012) binary
 * radix tree, boxes computed one tree depth at a time from the deepest, and a
 * four-wide view of the tree (each node's grandchildren) for the cone pass.
 * Enqueued on `stream`; returns after the build has finished (the call
 * synchronises `stream`).  Input arrays are not kept.  The copied indices and
 * coordinates are checked on the device first (host or device input alike):
 * an index outside [0, n_vertices) or a non-finite coordinate returns
 * VLS_ERR_INVALID_ARG and builds nothing. */
vls_status vls_scene_create(vls_context ctx, const vls_mesh_desc* mesh, void* stream, vls_scene* out);

/* One placement of a scene part (Sec. 3.5: a part may be loaded several times
 * and moved by transforms; Sec. 5.1: primitives rotate, scale and translate):
 * the part's vertices x map to A x + t, affine = the rows [A_i0 A_i1 A_i2 t_i],
 * i = 0..2 (row-major 3 x 4, float64, finite; any invertible or singular A). */
typedef struct {
    int32_t part;
    int32_t reserved;
    double affine[12];
} vls_instance_desc;

/* A scene of parts placed by instances.  Instance j contributes its part's
 * triangles with vertices evaluated in FP64 as ((A_i0 x + A_i1 y) + A_i2 z) +
 * t_i and rounded once to FP32, vertex indices offset by the instance's first
 * vertex, and the part's reflectance.  Instances are laid out in order: the
 * scene's triangle ids of instance j are [T_j, T_j + n_triangles of its part)
 * with T_j the triangles of the instances before it (vertices likewise), so a
 * hit id names its instance and its triangle in the part.  The result is then
 * built and traced exactly as vls_scene_create's (one LBVH over the placed
 * triangles; the device holds every placed copy).  Parts: as for
 * vls_scene_create, each with its own memory kind; a part index outside
 * [0, n_parts), a non-finite map, a part's vertex index outside its own
 * vertices or a non-finite placed vertex returns VLS_ERR_INVALID_ARG.  More
 * than 2^30 placed triangles or 2^31 placed vertices: VLS_ERR_UNSUPPORTED.
 * Synchronises `stream`. */
vls_status vls_scene_create_instanced(vls_context ctx, const vls_mesh_desc* parts, int32_t n_parts,
                                      const vls_instance_desc* instances, int32_t n_instances, void* stream,
                                      vls_scene* out);

/* The same scene kept in two levels: each part built once into its own LBVH in
 * its own frame, and a top-level LBVH over the instances' boxes in the scene's
 * frame (the part's box corners mapped in FP64 and rounded outward).  A subray
 * walks the top level, and in each instance it reaches walks the part's tree
 * with the ray mapped into the part's frame (A^-1 (O - t), A^-1 D: the ray
 * parameter stays the world distance), testing each leaf's triangle as placed
 * (the vertices of vls_scene_create_instanced, then the same world-frame
 * watertight test).  Hits, ids, distances, powers, waveforms and returns are
 * therefore those of the expanded scene, bit for bit, while the device holds
 * each part once.  Traced per subray (no cone pass): only vls_trace and
 * vls_simulate take such a scene (segments allowed; not in graphs, the
 * autotuner, the adjoint, vls_trace_counts, vls_cone_candidates or the scene
 * updates, voxels, specular materials and export, which return
 * VLS_ERR_UNSUPPORTED).  Maps must be invertible (VLS_ERR_UNSUPPORTED
 * otherwise); top-level depth <= 47 and part depth <= 63.  vls_simulate keeps
 * the subray arrays, waveform and window origins the caller leaves NULL in a
 * context workspace.  Synchronises `stream`. */
vls_status vls_scene_create_two_level(vls_context ctx, const vls_mesh_desc* parts, int32_t n_parts,
                                      const vls_instance_desc* instances, int32_t n_instances, void* stream,
                                      vls_scene* out);

/* New vertex positions (same count and triangles): leaf records and node boxes
 * are refitted, the tree topology is kept.  `vertices_dev` is a device array
 * [n_vertices][3] float32.  Asynchronous on `stream`. */
vls_status vls_scene_update_vertices(vls_scene scene, const float* vertices_dev, void* stream);

/* New per-triangle reflectance, device array [n_triangles] float32.  Asynchronous. */
vls_status vls_scene_update_reflectance(vls_scene scene, const float* reflectance_dev, void* stream);

/* A transmissive voxel grid (Sec. 3.5.4, Sec. 5.2): vegetation given as plant
 * area density (PAD, m^2/m^3) per voxel of an axis-aligned grid of cubes of
 * side voxel_size_m whose lowest corner is `origin`; voxel (ix, iy, iz) has
 * index ix + nx (iy + ny iz).  Model (the paper gives the equations; the
 * choices where it leaves room are stated here):
 *   sigma   = PAD * g(|v_z|), v the subray's unit direction; `lut` is the
 *             leaf-angle table (Table 2: hit probability against the beam's
 *             vertical component, whose horizontal component follows), rows of
 *             (vertical component, g), strictly increasing in the first; g is
 *             linear between rows and held beyond the first and last (Eq. 5's
 *             integral is what the table tabulates);
 *   depth   s = -ln(u) / sigma (Eq. 6), u uniform in (0, 1] from SplitMix64
 *             (Steele, Lea & Flood 2014) output number
 *             (pulse * 64 + subray) * (nx ny nz) + voxel of the sequence seeded
 *             with `seed`: u = ((x >> 11) + 1) 2^-53, one draw per voxel the
 *             subray crosses; `pulse` is the index in the call's pulse batch;
 *   stop    the subray stops in a voxel when s is at most the length it
 *             travels inside the voxel (Sec. 5.2), at s past its entry, and
 *             passes on otherwise (sigma = 0: always); voxels are visited in
 *             order along the subray (Amanatides & Woo 1987; Sec. 5.1's
 *             consecutive intersections without an epsilon step) and the nearer
 *             of the first stop and the closest triangle is the hit (a voxel
 *             stop at the triangle's distance wins);
 *   echo    subray_tri = n_triangles + voxel index, subray_cos = 1,
 *             subray_power = eta sigma P0 w D^2 / (4 pi R^4 beta^2) (Eq. 7 with
 *             the proportionality taken as equality; beta the full divergence,
 *             which must then be > 0); waveforms and returns take voxel echoes
 *             like triangle echoes, and ret_tri reports their ids alike.
 * pad [nz][ny][nx] float32 and lut [n_lut][2] float64 are HOST arrays, checked
 * (finite, PAD >= 0, g >= 0) and copied; the call synchronises `stream`.
 * n_triangles + nx ny nz must stay below 2^31.  A scene takes one grid, once
 * (a second call returns VLS_ERR_INVALID_ARG); graphs captured before the call
 * keep tracing without it.  vls_waveform_backward treats voxel echoes as
 * constants (they depend on neither reflectance nor vertices). */
typedef struct {
    double origin[3];
    double voxel_size_m;
    int32_t nx, ny, nz;
    int32_t n_lut;
    const float* pad;
    const double* lut;
    uint64_t seed;
} vls_voxel_desc;

vls_status vls_scene_set_voxels(vls_scene scene, const vls_voxel_desc* voxels, void* stream);

/* Specular materials (Sec. 5.1: primitives carry reflectance and specularity;
 * the paper gives no formula).  With them a triangle's surface response,
 * which takes the place of |cos theta| in the power of Eq. 7, is
 *   f = (1 - ks) |cos theta| + ks max(cos 2 theta, 0)^n,  cos 2 theta = 2 cos^2 theta - 1:
 * a Phong-type lobe for a receiver at the emitter, where the beam's mirror
 * direction makes the angle 2 theta with the way back; ks = 0 is Lambertian and
 * every ks returns f = 1 at normal incidence.  specularity_dev (ks, in [0, 1])
 * and exponent_dev (n >= 0) are device arrays [n_triangles] float32 by original
 * triangle index, copied asynchronously on `stream` into the scene (later calls
 * overwrite them in place, so graphs captured after the first call see new
 * values); both NULL turns the term off for later calls and captures.  The
 * library shades in FP32: the lobe multiplies the FP32 error of cos theta (a
 * few 2^-24) by about 4n + 3.  vls_waveform_backward differentiates f. */
vls_status vls_scene_set_specular(vls_scene scene, const float* specularity_dev, const float* exponent_dev,
                                  void* stream);

/* Synchronous: statistics of the built scene. */
vls_status vls_scene_stats_get(vls_scene scene, vls_scene_stats* out);

/* Synchronous debug copy of the structure to host memory (any pointer may be NULL):
 *   nodes      [n_internal_nodes][16] float32 words: left box lo.xyz hi.xyz,
 *              right box lo.xyz hi.xyz, then left ref, right ref, parent, 0 as
 *              int32 bits; a ref >= 0 is an internal node, ref < 0 is leaf ~ref
 *   leaf_tri   [n_triangles] int32: original triangle index of each leaf
 *   morton     [n_triangles] uint64: sorted Morton keys
 *   root       the root ref (0, or ~0 for a one-triangle scene, or -1 if empty) */
vls_status vls_scene_export(vls_scene scene, float* nodes, int32_t* leaf_tri, uint64_t* morton, int32_t* root);

vls_status vls_scene_destroy(vls_scene scene);

/* ------------------------------------------------------------------ scanner, pulses, outputs */

/* Instrument description (Sec. 3.4 subrays and waveform, Sec. 5.2 radar
 * equation, Sec. 5.4 bin size and window length).
 *   divergence_rad     full beam divergence at the 1/e^2 points
 *   n_subrays          1..64 subrays per pulse; 0 = use beam_quality.  Rings
 *                      i = 1, 2, ... hold floor(2 pi i) subrays (Sec. 3.4); a
 *                      count between ring totals fills rings in order and the
 *                      last ring holds the remainder, evenly spaced
 *   beam_quality       number of complete rings when n_subrays == 0
 *   pattern_extent     kappa: ring i of N at angle (i/N) kappa divergence/2
 *   pulse_shape        VLS_PULSE_GAUSSIAN (unit peak; width = FWHM) or
 *                      VLS_PULSE_EQ3 ((s/tau)^2 exp(-s/tau), tau = width/1.75)
 *   bin_ns, n_bins     the window samples t0 + j*bin_ns, j < n_bins (3..1024)
 *   window_pre_ns      t0 = first two-way travel time - window_pre_ns;
 *                      < 0 = automatic: 6 sigma (Gaussian) or 0 (Eq. 3)
 *   peak_power_w, receiver_diameter_m, efficiency
 *                      subray power P = peak * w_k * (eff * D^2 / 4) * rho * cos / R^2
 *                      (Eq. 7 with a Lambertian extended target)
 *   min_echo_abs, min_echo_rel
 *                      a return needs wf >= max(abs, rel * max wf)
 *   max_returns        K, 1..16 returns kept per pulse (the first K in time) */
typedef struct {
    double divergence_rad;
    double pattern_extent;
    double pulse_width_ns;
    double bin_ns;
    double window_pre_ns;
    double peak_power_w;
    double receiver_diameter_m;
    double efficiency;
    double min_echo_abs;
    double min_echo_rel;
    int32_t n_subrays;
    int32_t beam_quality;
    int32_t pulse_shape;
    int32_t n_bins;
    int32_t max_returns;
    int32_t reserved;
    double range_noise_m;   /* ranging error (Sec. 3.7): standard deviation in m, >= 0 (0: none) */
    uint64_t noise_seed;    /* its SplitMix64 seed */
} vls_scanner_desc;

/* Number of subrays the description yields (1..64), or an error for an
 * invalid description.  Host only; enqueues nothing. */
vls_status vls_scanner_subrays(const vls_scanner_desc* scanner, int32_t* n_subrays);

/* Pulses (the beam origin and direction recorded with each waveform, Sec. 3.6).
 *   origins        [n_pulses][3] float64, device
 *   directions     [n_pulses][3] float32, device; normalised in FP64 by the
 *                  library; a zero or non-finite direction makes every subray miss
 *   window_t0_ns   [n_pulses] float64, device, or NULL: fixed window origins
 *                  (NaN = no window; used to hold t0 fixed for gradients)
 *   segment_offsets [n_segments+1] int64, HOST, or NULL: pulses of segment s
 *                  are [off[s], off[s+1]); off[0] = 0, off[n] = n_pulses
 *   segment_scanner [n_segments] int32, HOST: index into the scanner array
 * Without segments every pulse uses scanners[0]. */
typedef struct {
    const double* origins;
    const float* directions;
    const double* window_t0_ns;
    int64_t n_pulses;
    const int64_t* segment_offsets;
    const int32_t* segment_scanner;
    int32_t n_segments;
    int32_t reserved;
} vls_pulse_batch;

/* Outputs, all device arrays owned by the caller; any may be NULL unless a
 * function needs it.  S_stride = the largest subray count of the scanners in
 * the call; per-subray arrays are [n_pulses][S_stride] (unused tail entries of
 * a pulse with fewer subrays are left untouched).
 *   subray_tri      int32, hit triangle (original index) or -1 for a miss
 *   subray_range    float64, metres (+inf for a miss)
 *   subray_cos      float32, |cos| of the incidence angle (0 for a miss)
 *   subray_power    float32, watts (0 for a miss)
 *   waveform        [n_pulses][n_bins] float32
 *   window_t0_ns    [n_pulses] float64 (NaN when no subray hit)
 *   n_returns       [n_pulses] int32
 *   ret_range       [n_pulses][K] float32 metres: (c/2)(t0 + j*bin - s_peak)
 *   ret_amplitude   [n_pulses][K] float32, waveform value at the return's bin
 *   ret_tri         [n_pulses][K] int32, triangle of the subray contributing
 *                   most at that bin (lowest subray index on ties)
 *   ret_bin         [n_pulses][K] int32
 * Slots past n_returns hold range 0, amplitude 0, tri -1, bin -1. */
typedef struct {
    int32_t* subray_tri;
    double* subray_range;
    float* subray_cos;
    float* subray_power;
    float* waveform;
    double* window_t0_ns;
    int32_t* n_returns;
    float* ret_range;
    float* ret_amplitude;
    int32_t* ret_tri;
    int32_t* ret_bin;
} vls_outputs;

/* ------------------------------------------------------------------ the hot path */

/* Subrays and closest hits only (Sec. 3.4 first hit; Sec. 5.1 minimum-distance
 * intersection).  Writes subray_tri (required), subray_range, subray_cos,
 * subray_power.  Ties on equal distance go to the lower triangle index;
 * triangle edges are inclusive; only distances > 0 count. */
vls_status vls_trace(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                     const vls_pulse_batch* pulses, const vls_outputs* out, void* stream);

/* Waveform synthesis from traced subrays (Sec. 3.4, Eq. 3): reads subray_tri,
 * subray_range, subray_power; writes waveform (required) and window_t0_ns. */
vls_status vls_waveform(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, void* stream);

/* Returns from waveforms (Sec. 3.4 local maxima): reads waveform and
 * window_t0_ns; writes n_returns, ret_range, ret_amplitude, ret_bin (required)
 * and ret_tri, which needs subray_tri, subray_range and subray_power (if they
 * are NULL, ret_tri is -1). */
vls_status vls_returns(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                       const vls_pulse_batch* pulses, const vls_outputs* out, void* stream);

/* ------------------------------------------------------------------ surveys */

/* Scan deflectors (Sec. 3.3, Fig. 7) and platforms (Sec. 3.2). */
enum { VLS_DEFLECT_POLYGON = 0, VLS_DEFLECT_SWING = 1, VLS_DEFLECT_CONIC = 2, VLS_DEFLECT_FIBRE = 3 };
enum { VLS_PLATFORM_LINEAR = 0, VLS_PLATFORM_MULTICOPTER = 1, VLS_PLATFORM_MULTICOPTER_SMOOTH = 2 };

/* A survey: a platform (Sec. 3.2) carrying a scanner with a deflector (Sec.
 * 3.3).  The paper gives the platforms' and deflectors' behaviour but no
 * formulas; the model:
 *   pulse k leaves at t = t0_s + k / pulse_rate_hz;
 *   LinearPath platform (n_waypoints >= 2): covers the polyline at speed_mps
 *   from the first waypoint at t = 0, level, facing the current leg's
 *   horizontal direction, and stays at the last waypoint afterwards; one
 *   waypoint: static, facing +x;
 *   Multicopter platform (it also speeds up and slows down; the mode without
 *   banked turns, which stops and turns at each waypoint): every leg starts
 *   from rest and ends at rest, accelerating at accel_mps2 up to speed_mps,
 *   holding it, and slowing down at the same rate (a leg shorter than
 *   speed^2 / accel speeds up over its first half and slows down over its
 *   second); turns take no time; level; yaw is the leg's heading, or, with
 *   leg_yaw, linear in the time on the leg from its start to its end value;
 *   Multicopter platform with smooth turns (it banks to turn at the
 *   waypoints instead of stopping there): a coordinated turn at each interior
 *   waypoint on the circular arc tangent to both legs, of radius
 *   r = v^2 / (g tan b) (v = speed_mps, b = bank_angle_rad, g = 9.80665 m/s^2),
 *   from W - s u to W + s w (u, w the unit directions into and out of W,
 *   s = r tan(theta / 2), theta = acos(u . w)), in the plane of the two legs;
 *   from rest at the first waypoint it speeds up at accel_mps2 to v, keeps v
 *   along the straight parts and the arcs, and slows down to rest at the last
 *   waypoint, where it stays; heading along the horizontal direction of
 *   motion; level on the straight parts, banked by b toward the turn's centre
 *   on an arc (a platform direction (x, y, z) becomes
 *   (x, y cos l + z sin l, -y sin l + z cos l), l = +b for a turn to the left,
 *   -b to the right, before the heading); every leg must hold its arcs (s at
 *   each end) and, on the first and the last leg, the ramp v^2 / (2 accel),
 *   no turn may exceed 179 degrees, and leg_yaw must be NULL;
 *   platform frame x forward, y left, z up; with A = scan_angle_rad and
 *   f = scan_freq_hz the beam points along (0, sin a, -cos a) with
 *     POLYGON a = -A + 2A frac(f t)        (parallel lines, even density)
 *     SWING   a = A sin(2 pi f t)          (zig-zag, denser at the extremes)
 *     FIBRE   a = -A + 2A (k mod n_fibres) / (n_fibres - 1)
 *   or, CONIC (Palmer), along (sin A cos p, sin A sin p, -cos A), p = 2 pi frac(f t);
 *   platform_noise_m > 0 adds independent N(0, sigma^2) offsets per axis to
 *   each origin, from SplitMix64 (Steele, Lea & Flood 2014) outputs
 *   6k + 2 axis and 6k + 2 axis + 1 of the sequence seeded with `seed`
 *   (Box-Muller), so any range of pulses can be generated on its own.
 * waypoints: [n_waypoints][3] float64 in host memory, finite, consecutive ones
 * distinct; copied, as is leg_yaw (the library caches one device table per
 * distinct survey). */
typedef struct {
    const double* waypoints;
    int32_t n_waypoints;
    int32_t deflector;
    double speed_mps;
    double pulse_rate_hz;
    double scan_freq_hz;
    double scan_angle_rad;
    int32_t n_fibres;
    int32_t platform;          /* VLS_PLATFORM_*; 0 (LinearPath) for older callers */
    double t0_s;
    double platform_noise_m;
    uint64_t seed;
    double accel_mps2;         /* Multicopter: > 0 (with speed_mps > 0) when n_waypoints >= 2 */
    const double* leg_yaw;     /* Multicopter: NULL, or host [n_waypoints - 1][2] start and end
                                  yaw (rad, finite) of each leg; NULL for the other platforms */
    double bank_angle_rad;     /* Multicopter with smooth turns: bank angle in (0, pi/2) */
} vls_survey_desc;

/* Pulses [first, first + count) of a survey, on the device, in the layout
 * vls_simulate takes: origins [count][3] float64, directions [count][3]
 * float32 (unit), both device arrays.  Enqueued on `stream` (the first call
 * with a new survey uploads its table synchronously).  Errors:
 * VLS_ERR_INVALID_ARG for an invalid survey, a negative range or missing or
 * misaligned outputs. */
vls_status vls_generate_pulses(vls_context ctx, const vls_survey_desc* survey, int64_t first, int64_t count,
                               double* origins, float* directions, void* stream);

/* Echo width (Sec. 3.4: an optional Gaussian fitted by non-linear least squares
 * to the waveform of each return, whose standard deviation is the return's
 * width; the return's position stays the local maximum).  For every kept
 * return of every pulse, the samples are the return's lobe: from the return's
 * bin outward while the waveform keeps falling strictly and stays at or above
 * 2^-10 of the return bin's value, at most 31 bins to each side.  The model
 * A exp(-(x - mu)^2 / (2 s^2)) starts from the Gaussian through the return's
 * bin and its two neighbours (when they lie in the lobe, are positive and curve
 * downward), else from the bin's value and the pulse's own standard deviation,
 * and is fitted by 12 Levenberg-Marquardt iterations in FP32 (trial points
 * centred farther out than the lobe is long, or wider than twice its bins,
 * count as rejected).
 *   reads    out->waveform, out->n_returns, out->ret_bin (as vls_simulate or
 *            vls_returns wrote them; the other output arrays are not used)
 *   width_ns device array [n_pulses][K] float32: |s| in ns for the kept
 *            returns, NaN where no fit exists (a lobe of fewer than three bins,
 *            a fit ending with A <= 0) and for the slots past n_returns.
 * The context keeps a workspace of n_pulses * K ints, grown on demand.  Enqueued
 * on `stream`.  Errors: VLS_ERR_INVALID_ARG for missing arrays, as vls_returns
 * for the scanners and the batch. */
vls_status vls_echo_width(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                          const vls_pulse_batch* pulses, const vls_outputs* out, float* width_ns, void* stream);

/* The whole path fused in one launch: trace, power, waveform, returns.
 * waveform may be NULL (returns are still found from the in-register
 * waveform, Sec. 5.4: binning runs even when no waveform is written).
 * With segments, one launch per scanner covers its segments (or, with the
 * launch configuration's grouped = 0, one persistent launch covers them all).
 * Before it, a
 * cone pass lists each pulse's candidate triangles (Sec. 3.4: every subray of
 * a pulse leaves its origin within the beam's divergence): up to
 * VLS_MAX_CANDIDATES per pulse in the stream's workspace (1 KiB per pulse);
 * a pulse whose walk reaches more than 159 gets a second walk into a long list
 * of up to 1,024 (4 KiB each, for the first 262,144 such pulses of a call);
 * a pulse past that is walked by one wavefront, all its subrays together.
 * The results do not depend on which of these a pulse takes. */
vls_status vls_simulate(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, void* stream);

/* vls_simulate for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same kernels as vls_simulate on one scanner (results equal to its own), but
 * every workspace lives in a fixed device array of the library's, which each
 * GPU the library runs on holds until the process ends: the scanner's subray
 * table (stored by a small kernel, the table travelling as its argument) and
 * the cone pass's candidate lists, overflow list, counters and pulse bases
 * (VLS_NOALLOC_SCRATCH_BYTES bytes).  The call makes no hipMalloc, hipFree or
 * other allocating call and records no timing events; the caller still passes
 * the inputs and outputs.
 *   scanner   one description (no segments: pulses->n_segments must be 0)
 *   pulses    n_pulses <= VLS_NOALLOC_MAX_PULSES; larger batches are split by
 *             the caller
 *   scene     a scene from vls_scene_create or vls_scene_create_instanced (not
 *             two-level)
 * Every call on a GPU shares that GPU's array, and each call rewrites what it
 * reads there before reading it (the counters with a fill kernel), so
 * consecutive calls on one stream are independent.  Calls that overlap on one
 * GPU (other streams, other contexts or threads) race on the array and must be
 * ordered by the caller.
 * Errors: as vls_simulate; VLS_ERR_INVALID_ARG for more than
 * VLS_NOALLOC_MAX_PULSES pulses; VLS_ERR_UNSUPPORTED for segments or a
 * two-level scene; VLS_ERR_DEVICE if the array's address could not be found
 * when the context was created. */
#define VLS_NOALLOC_MAX_PULSES 32768
#define VLS_NOALLOC_SCRATCH_BYTES (2560 + 4 * (267 * 32768 + 4))
vls_status vls_simulate_noalloc(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanner,
                                const vls_pulse_batch* pulses, const vls_outputs* out, void* stream);

/* ------------------------------------------------------------------ adjoint */

/* Gradient of a waveform loss L with respect to per-triangle reflectance and
 * vertex heights (z), given G = dL/dwf.  Hit selection is held fixed (the
 * forward's subray_tri), the window origins are the fixed window_t0_ns of
 * `pulses` (required), and each subray's range, incidence and power are
 * recomputed from the scene's current vertices and reflectance (Sec. 5.2,
 * Eq. 7; Sec. 3.4, Eq. 3): dL/drho, and dL/dz through R = n.(a-O)/(n.d),
 * cos = |n.d|/|n| and P = C w rho cos / R^2.
 *   scanner            one description; no segments
 *   subray_tri         [n_pulses][S] int32 device, from vls_simulate/vls_trace
 *   grad_waveform      [n_pulses][n_bins] float32 device
 *   grad_reflectance   [n_triangles] float32 device, overwritten (may be NULL)
 *   grad_vertex_z      [n_vertices] float32 device, overwritten (may be NULL)
 * By default each wavefront sums the contributions of its subrays that share a
 * triangle and adds them with float atomics, so the summation order, and the
 * last bits, vary between runs.  With vls_set_deterministic(ctx, 1) every
 * subray's contributions are written as entries keyed by their parameter
 * (triangle or vertex), stably sorted by key, and each parameter's entries
 * summed in subray order in FP64: bitwise repeatable, at the cost of a
 * workspace of 112 B per subray (grown on the stream) and a radix sort.
 * Asynchronous on `stream`. */
vls_status vls_waveform_backward(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanner,
                                 const vls_pulse_batch* pulses, const int32_t* subray_tri, const float* grad_waveform,
                                 float* grad_reflectance, float* grad_vertex_z, void* stream);

/* Summation order of vls_waveform_backward: 0 (default) wavefront sums and
 * float atomics; 1 a fixed order (sort by parameter, sums in subray order), so
 * two runs on the same inputs give bitwise equal gradients. */
vls_status vls_set_deterministic(vls_context ctx, int32_t on);

/* ------------------------------------------------------------------ launch configuration */

typedef struct {
    int32_t block_waves;       /* wavefronts per block: 1, 2, 4 (default 1)                      */
    int32_t stack_lds;         /* traversal-stack entries per lane held in LDS: 4, 8, 16, 32
                                  (default 16); deeper entries spill to per-lane scratch          */
    int32_t persistent_blocks; /* blocks of the persistent kernel; 0 = auto (CUs x occupancy)    */
    int32_t pack;              /* 0: floor(64/S) pulses per wavefront; 1: one pulse per wavefront */
    int32_t cone;              /* 1 (default): one cone traversal per pulse collects the triangles
                                  its subrays can hit (same results, less work); 0: every subray
                                  traverses the LBVH on its own                                    */
    int32_t cover_off;         /* 0 (default): the cone traversal culls the triangles behind one
                                  that covers the whole beam (an FP64 test of leaves on its way);
                                  1: it does not (shorter walks, longer candidate lists, the same
                                  results): faster where candidates are cheap to test, as for
                                  vegetation scanned with one pulse per wavefront               */
    int32_t grouped;           /* batches (segments): 1 (default) one launch per scanner over its
                                  segments' wavefront tiles, each the fused kernel of that
                                  scanner's layout; 0 one persistent launch for all segments,
                                  whose wavefronts take tiles from a work counter (same results)  */
    int32_t reserved;
} vls_launch_config;

vls_status vls_set_launch_config(vls_context ctx, const vls_launch_config* cfg);
vls_status vls_get_launch_config(vls_context ctx, vls_launch_config* cfg);

/* Diagnostic, synchronous: traces the batch (nothing is written to outputs)
 * and stores in counts[0..2] the number of subrays traced, internal-node
 * visits and triangle tests of the traversal.  These give the algorithmic
 * bytes of the path: 64 B per node visit and 48 B per triangle test. */
vls_status vls_trace_counts(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                            const vls_pulse_batch* pulses, uint64_t* counts, void* stream);

/* ------------------------------------------------------------------ batched form: graphs and tuning */

/* Captures the whole vls_simulate call (counter reset + launch) into a HIP
 * graph on a private stream.  Every pointer in `pulses` and `out` is baked
 * into the graph and must stay valid until vls_graph_destroy; the host
 * segment arrays are copied at capture.  The launch configuration of `ctx` at
 * capture time is used.  Replays of one graph must not overlap in time. */
vls_status vls_graph_capture(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                             const vls_pulse_batch* pulses, const vls_outputs* out, vls_graph* graph);
vls_status vls_graph_launch(vls_graph graph, void* stream);
vls_status vls_graph_destroy(vls_graph graph);

typedef struct {
    vls_launch_config best;
    double best_ms;            /* time of one vls_simulate call with `best`                 */
    double default_ms;         /* time with the configuration the context had on entry      */
    int32_t n_tried;           /* configurations timed (0 when taken from the cache)        */
    int32_t from_cache;
} vls_tune_result;

/* Times vls_simulate on this batch for launch configurations (block shape,
 * LDS stack depth, pulses per wavefront, persistent grid size, cone pass on or
 * off, its cover tests on or off, grouped or persistent batches) by
 * coordinate descent with HIP events on `stream` (a configuration's time: the
 * fastest of three pairs of calls after one warm-up call), keeps the fastest in
 * `ctx`, and appends
 * it to `cache_path` (JSON lines, may be NULL) keyed by scene size, subray
 * counts, bins, pulse count and segments.  A matching cache entry is used
 * without timing.  Writes the outputs as vls_simulate does.  Synchronous. */
vls_status vls_autotune(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, const char* cache_path, void* stream,
                        vls_tune_result* result);

/* Diagnostic: runs only the cone pass (the per-pulse traversal that collects
 * the triangles a pulse's subrays can hit) into `candidates`, a device array
 * [n_pulses][VLS_MAX_CANDIDATES + 1] int32: entry 0 is the count (-1 when more
 * than VLS_MAX_CANDIDATES triangles were reached and the subrays traverse on
 * their own), then the original triangle indices.  Asynchronous on `stream`. */
vls_status vls_cone_candidates(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners,
                               int32_t n_scanners, const vls_pulse_batch* pulses, int32_t* candidates, void* stream);

/* Kernel timing for measurement (no passage of the paper: it instruments the
 * calls above).  While enabled, every eager vls_simulate call records a pair of
 * HIP events on its stream around the cone pass, around the packet walk of the
 * pulses whose candidate list overflowed, and around the fused kernel (or the
 * batch's launches); nothing is recorded while the stream is being captured
 * into a graph.  vls_profile_read waits for the recorded events, returns the
 * summed elapsed times and launch counts since the previous read, and clears
 * them.  The events are owned by the context.  Errors: VLS_ERR_INVALID_ARG for
 * NULL arguments; a failed event call returns VLS_ERR_DEVICE. */
typedef struct {
    double cone_ms;          /* summed over the recorded cone passes          */
    double fused_ms;         /* summed over the recorded fused kernels        */
    int64_t cone_launches;
    int64_t fused_launches;
    double packet_ms;        /* summed over the recorded packet walks (pulses
                                whose candidate list overflowed)              */
    int64_t packet_launches;
} vls_profile;
vls_status vls_profile_enable(vls_context ctx, int32_t enable);
vls_status vls_profile_read(vls_context ctx, vls_profile* out);

/* Synchronise `stream` and report any device error as VLS_ERR_DEVICE. */
vls_status vls_synchronize(vls_context ctx, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VLS_H */
