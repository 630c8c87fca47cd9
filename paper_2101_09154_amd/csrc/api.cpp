// Host runtime behind the C ABI declared in include/vls.h: argument
// validation, per-scanner subray tables, scene lifecycle and kernel dispatch.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "vls.h"
#include "vls_internal.h"

using namespace vls;

namespace {

thread_local std::string g_err;

vls_status fail(vls_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

vls_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VLS_ERR_OUT_OF_MEMORY : VLS_ERR_DEVICE;
}

#define VLS_HIP(call, what)                            \
    do {                                               \
        hipError_t e__ = (call);                       \
        if (e__ != hipSuccess) return hip_fail(e__, what); \
    } while (0)

// ------------------------------------------------------------------ subray table (Sec. 3.4)

int ring_capacity(int i) { return (int)std::floor(2.0 * M_PI * (double)i); }

// Ring sizes: complete rings 1..quality, or ring-fill to n_subrays.
bool ring_sizes(int n_subrays, int quality, std::vector<int>& rings)
{
    rings.clear();
    if (n_subrays <= 0) {
        if (quality < 0 || quality > 64) return false;
        for (int i = 1; i <= quality; ++i) rings.push_back(ring_capacity(i));
        return true;
    }
    int left = n_subrays - 1;
    for (int i = 1; left > 0; ++i) {
        int m = std::min(ring_capacity(i), left);
        rings.push_back(m);
        left -= m;
    }
    return true;
}

// table[k] = {cos a, sin a, cos phi, sin phi, w}: central subray, then rings
// outward; ring i of N at a = (i/N) kappa div/2, phi = 2 pi m / n_i; w from the
// Gaussian beam profile (Eq. 1, far field: r/w = tan a / tan(div/2)), sum 1.
int subray_table(const vls_scanner_desc& d, std::vector<double>& table)
{
    std::vector<int> rings;
    if (!ring_sizes(d.n_subrays, d.beam_quality, rings)) return -1;
    int S = 1;
    for (int m : rings) S += m;
    if (S > VLS_MAX_SUBRAYS) return -S;
    const int N = (int)rings.size();
    const double half = 0.5 * d.divergence_rad, th = std::tan(half);
    std::vector<double> al(S), ph(S), w(S);
    int k = 0;
    al[k] = 0.0;
    ph[k] = 0.0;
    ++k;
    for (int i = 1; i <= N; ++i)
        for (int m = 0; m < rings[i - 1]; ++m, ++k) {
            al[k] = ((double)i / (double)N) * (d.pattern_extent * half);
            ph[k] = 2.0 * M_PI * (double)m / (double)rings[i - 1];
        }
    double sum = 0.0;
    for (k = 0; k < S; ++k) {
        double x = th > 0.0 ? std::tan(al[k]) / th : 0.0;
        w[k] = std::exp(-2.0 * x * x);
        sum += w[k];
    }
    table.resize(5 * (size_t)S);
    for (k = 0; k < S; ++k) {
        table[5 * k + 0] = std::cos(al[k]);
        table[5 * k + 1] = std::sin(al[k]);
        table[5 * k + 2] = std::cos(ph[k]);
        table[5 * k + 3] = std::sin(ph[k]);
        table[5 * k + 4] = w[k] / sum;
    }
    return S;
}

bool finite_pos(double x) { return x > 0.0 && std::isfinite(x); }

vls_status check_scanner(const vls_scanner_desc& d, int idx)
{
    char b[160];
    auto bad = [&](const char* what) {
        snprintf(b, sizeof b, "scanner %d: %s", idx, what);
        return fail(VLS_ERR_INVALID_ARG, b);
    };
    if (!(d.divergence_rad >= 0.0) || !std::isfinite(d.divergence_rad)) return bad("divergence_rad must be finite and >= 0");
    if (!(d.range_noise_m >= 0.0) || !std::isfinite(d.range_noise_m)) return bad("range_noise_m must be finite and >= 0");
    if (!(d.pattern_extent >= 0.0) || !std::isfinite(d.pattern_extent)) return bad("pattern_extent must be finite and >= 0");
    if (!finite_pos(d.pulse_width_ns)) return bad("pulse_width_ns must be > 0");
    if (!finite_pos(d.bin_ns)) return bad("bin_ns must be > 0");
    if (d.n_bins < 3 || d.n_bins > VLS_MAX_BINS) return bad("n_bins must be in [3, 1024]");
    if (d.max_returns < 1 || d.max_returns > VLS_MAX_RETURNS) return bad("max_returns must be in [1, 16]");
    if (d.pulse_shape != VLS_PULSE_GAUSSIAN && d.pulse_shape != VLS_PULSE_EQ3) return bad("unknown pulse_shape");
    if (d.n_subrays < 0 || d.n_subrays > VLS_MAX_SUBRAYS) return bad("n_subrays must be in [0, 64]");
    if (d.n_subrays == 0 && d.beam_quality < 0) return bad("beam_quality must be >= 0");
    if (!std::isfinite(d.window_pre_ns)) return bad("window_pre_ns must be finite");
    if (!std::isfinite(d.peak_power_w) || !std::isfinite(d.receiver_diameter_m) || !std::isfinite(d.efficiency))
        return bad("radiometric constants must be finite");
    if (!std::isfinite(d.min_echo_abs) || !std::isfinite(d.min_echo_rel)) return bad("echo thresholds must be finite");
    std::vector<int> rings;
    if (!ring_sizes(d.n_subrays, d.beam_quality, rings)) return bad("bad subray request");
    int S = 1;
    for (int m : rings) S += m;
    if (S > VLS_MAX_SUBRAYS) {
        snprintf(b, sizeof b, "scanner %d: %d subrays exceed %d (one wavefront per pulse)", idx, S, VLS_MAX_SUBRAYS);
        return fail(VLS_ERR_UNSUPPORTED, b);
    }
    return VLS_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

// ------------------------------------------------------------------ objects

struct vls_context_s {
    int device = 0;
    LaunchCfg cfg;
    std::map<std::string, double*> patterns;  // subray tables on the device
    struct Batch {
        std::vector<unsigned char> key;
        unsigned char* dev = nullptr;
        BatchDev bd;
        std::vector<GroupDev> groups;  // per scanner: its segments, for grouped launches
        int max_bins = 0;
    };
    std::vector<Batch> batches;  // uploaded segment tables (read-only), reused by content
    // Per-stream workspaces: every stream the context is used with gets its own,
    // grown on demand by stream-ordered allocations on that stream, so calls on
    // different streams never share scratch memory and growing one waits for
    // nothing but earlier work on its own stream.
    struct Workspace {
        hipStream_t stream = nullptr;
        int* cand = nullptr;                // cone-pass workspace (cone_ws_*)
        size_t cand_bytes = 0;
        int* longw = nullptr;               // long candidate lists (long_ws_*)
        size_t long_bytes = 0;
        int* ew = nullptr;                  // echo-width list of returns + counter
        size_t ew_bytes = 0;
        unsigned char* tlw = nullptr;       // two-level simulate: subrays, waveform and t0 not asked for
        size_t tlw_bytes = 0;
        unsigned char* adw = nullptr;       // adjoint in fixed summation order: entries and sort buffers
        size_t adw_bytes = 0;
        unsigned long long* ctr = nullptr;  // the batched launch's work counter
        size_t ctr_bytes = 0;
    };
    std::vector<std::unique_ptr<Workspace>> workspaces;
    bool deterministic = false;  // the adjoint sums in a fixed order (vls_set_deterministic)
    struct SurveyTab {
        std::vector<double> key;   // the host table it was made from
        double* dev = nullptr;
    };
    std::vector<SurveyTab> surveys;  // device waypoint tables, one per distinct survey
    void* noalloc_ptr = nullptr;     // this device's scratch of vls_simulate_noalloc
    hipError_t noalloc_status = hipSuccess;
    // kernel timing (vls_profile_*): event pairs recorded around the cone pass
    // and the fused kernel of eager vls_simulate calls, and a pool of spares
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_cone, prof_packets, prof_fused, prof_pool;
    ~vls_context_s()
    {
        (void)hipSetDevice(device);
        for (auto* v : {&prof_cone, &prof_packets, &prof_fused, &prof_pool})
            for (auto& e : *v) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        for (auto& w : workspaces)
            for (void* q : {(void*)w->cand, (void*)w->longw, (void*)w->ew, (void*)w->tlw, (void*)w->adw, (void*)w->ctr})
                if (q) (void)hipFreeAsync(q, nullptr);
        (void)hipDeviceSynchronize();
        for (auto& t : surveys) (void)hipFree(t.dev);
        for (auto& kv : patterns) (void)hipFree(kv.second);
        for (auto& b : batches) (void)hipFree(b.dev);
    }
};

struct vls_scene_s;

// A two-level scene: each part's own scene (its LBVH in its own frame), the
// top-level scene over the instances' boxes, and the device tables.
struct TwoLevelHost {
    std::vector<vls_scene_s*> parts;   // by part index (null: unused or empty)
    vls_scene_s* top = nullptr;
    InstDev* inst = nullptr;           // [n_inst] in top-level leaf order
    PartDev* parts_dev = nullptr;
    TwoLevelDev dev{};
    ~TwoLevelHost();
};

struct vls_scene_s {
    std::unique_ptr<TwoLevelHost> tl;  // set for a two-level scene (b is then empty)
    vls_context ctx = nullptr;
    BvhBuffers b;
    vls_scene_stats stats{};
    int root = -1;
    VoxDev vox{};              // transmissive voxel grid (n_vox == 0: none); arrays owned here
    float* spec = nullptr;     // [2][n_tri]: specularity, then Phong exponent (allocated on first use)
    bool spec_on = false;
    ~vls_scene_s()
    {
        (void)hipFree(spec);
        (void)hipFree(const_cast<float*>(vox.pad));
        (void)hipFree(const_cast<double*>(vox.lut));
        (void)hipFree(b.nodes);
        (void)hipFree(b.nodes4);
        (void)hipFree(b.tris);
        (void)hipFree(b.refl);
        (void)hipFree(b.verts);
        (void)hipFree(b.tri_idx);
        (void)hipFree(b.leaf_parent);
        (void)hipFree(b.node_parent);
        (void)hipFree(b.leaf_tri);
        (void)hipFree(b.morton);
        (void)hipFree(b.node_depth);
        (void)hipFree(b.level_order);
        (void)hipFree(b.bounds);
    }
};

TwoLevelHost::~TwoLevelHost()
{
    for (vls_scene_s* p : parts) delete p;
    delete top;
    (void)hipFree(inst);
    (void)hipFree(parts_dev);
}

struct vls_graph_s {
    vls_context ctx = nullptr;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int* cand = nullptr;                // the graph's own cone-pass workspace,
    int* longw = nullptr;               // long candidate lists
    unsigned long long* ctr = nullptr;  // and its own work counter for a batched launch
    ~vls_graph_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        (void)hipFree(cand);
        (void)hipFree(longw);
        (void)hipFree(ctr);
    }
};

namespace {

// Everything of a scanner's device description but its subray table's device
// copy (s.pattern stays null); the table itself goes to `table`.
vls_status scanner_params(vls_context ctx, const vls_scanner_desc& d, ScannerDev& s, std::vector<double>& table)
{
    int S = subray_table(d, table);
    if (S <= 0) return fail(VLS_ERR_UNSUPPORTED, "subray pattern too large");
    memset(&s, 0, sizeof s);
    s.S = S;
    s.P_w = ctx->cfg.pack ? 1 : kWave / S;
    s.n_bins = d.n_bins;
    s.K = d.max_returns;
    s.shape = d.pulse_shape;
    s.bin_ns = (float)d.bin_ns;
    s.bin_d = d.bin_ns;
    s.inv_bin = (float)(1.0 / d.bin_ns);
    const double log2e = 1.4426950408889634;
    if (d.pulse_shape == VLS_PULSE_GAUSSIAN) {
        double sg = d.pulse_width_ns / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        s.neg_k = (float)(-log2e / (2.0 * sg * sg));
        s.inv_tau = 0.0f;
        // beyond 6.5 sigma the pulse is below 1e-9 of its peak
        s.cut_lo = (float)(6.5 * sg);
        s.cut_hi = (float)(6.5 * sg);
        s.t_pre = d.window_pre_ns < 0.0 ? 6.0 * sg : d.window_pre_ns;
        s.s_peak = 0.0;
    } else {
        double tau = d.pulse_width_ns / 1.75;
        s.neg_k = (float)(-log2e);
        s.inv_tau = (float)(1.0 / tau);
        // beyond 29 tau, (s/tau)^2 exp(-s/tau) is below 1e-9 of its peak 4 exp(-2)
        s.cut_lo = 0.0f;
        s.cut_hi = (float)(29.0 * tau);
        s.t_pre = d.window_pre_ns < 0.0 ? 0.0 : d.window_pre_ns;
        s.s_peak = 2.0 * tau;
    }
    s.power_c = d.peak_power_w * d.efficiency * d.receiver_diameter_m * d.receiver_diameter_m / 4.0;
    s.vox_c = s.power_c / (M_PI * d.divergence_rad * d.divergence_rad);
    s.tan_max = S > 1 ? std::tan(d.pattern_extent * 0.5 * d.divergence_rad) : 0.0;
    s.range_noise = d.range_noise_m;
    s.noise_seed = d.noise_seed;
    s.thr_abs = d.min_echo_abs;
    s.thr_rel = d.min_echo_rel;
    return VLS_OK;
}

// The scanner's device description with its subray table uploaded once per
// context and distinct table.
vls_status scanner_dev(vls_context ctx, const vls_scanner_desc& d, ScannerDev& s)
{
    std::vector<double> table;
    vls_status st = scanner_params(ctx, d, s, table);
    if (st != VLS_OK) return st;
    char key[160];
    snprintf(key, sizeof key, "%d|%a|%a", s.S, d.divergence_rad, d.pattern_extent);
    double* dev = nullptr;
    auto it = ctx->patterns.find(key);
    if (it == ctx->patterns.end()) {
        VLS_HIP(hipMalloc(&dev, sizeof(double) * table.size()), "pattern alloc");
        hipError_t e = hipMemcpy(dev, table.data(), sizeof(double) * table.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dev);
            return hip_fail(e, "pattern upload");
        }
        ctx->patterns[key] = dev;
    } else {
        dev = it->second;
    }
    s.pattern = dev;
    return VLS_OK;
}

SceneDev scene_dev(vls_scene sc)
{
    SceneDev s;
    s.nodes = sc->b.nodes;
    s.nodes4 = sc->b.nodes4;
    s.tris = sc->b.tris;
    s.refl = sc->b.refl;
    s.bounds = sc->b.bounds;
    s.verts = sc->b.verts;
    s.tri_idx = sc->b.tri_idx;
    s.root = sc->root;
    s.n_tri = (int)sc->b.n_tri;
    s.vox = sc->vox;
    s.spec_k = sc->spec_on ? sc->spec : nullptr;
    s.spec_n = sc->spec_on ? sc->spec + sc->b.n_tri : nullptr;
    return s;
}

struct Prepared {
    std::vector<ScannerDev> sc;
    int S_stride = 1;
    int n_bins = 0, K = 0;
    bool same_layout = true;
    std::vector<int64_t> off;   // segment offsets (or {0, n})
    std::vector<int32_t> seg_sc;
};

// The most candidate records any of the scanners stages in LDS per wavefront
// (pulses per wavefront times staged_per_pulse), or 0.
int staged_slots(const Prepared& pr)
{
    int m = 0;
    for (const auto& s : pr.sc) m = std::max(m, s.P_w * staged_per_pulse(s.P_w));
    return m;
}

// tables: when not null, the scanners' subray tables are left on the host
// (appended here, one per scanner) and no device table is uploaded.
vls_status prepare(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners, const vls_pulse_batch* pulses,
                   Prepared& pr, std::vector<std::vector<double>>* tables = nullptr)
{
    if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
    if (!scanners || n_scanners < 1 || n_scanners > VLS_MAX_SCANNERS)
        return fail(VLS_ERR_INVALID_ARG, "need 1..64 scanner descriptions");
    if (!pulses) return fail(VLS_ERR_INVALID_ARG, "pulse batch is NULL");
    if (pulses->n_pulses < 0) return fail(VLS_ERR_INVALID_ARG, "n_pulses < 0");
    if (pulses->n_pulses > 0 && (!pulses->origins || !pulses->directions))
        return fail(VLS_ERR_INVALID_ARG, "origins and directions are required");
    if (!aligned(pulses->origins, 8) || !aligned(pulses->directions, 4) || !aligned(pulses->window_t0_ns, 8))
        return fail(VLS_ERR_INVALID_ARG, "misaligned pulse arrays");
    pr.sc.resize(n_scanners);
    for (int i = 0; i < n_scanners; ++i) {
        vls_status st = check_scanner(scanners[i], i);
        if (st != VLS_OK) return st;
        if (tables) {
            tables->emplace_back();
            st = scanner_params(ctx, scanners[i], pr.sc[i], tables->back());
        } else {
            st = scanner_dev(ctx, scanners[i], pr.sc[i]);
        }
        if (st != VLS_OK) return st;
    }
    pr.n_bins = pr.sc[0].n_bins;
    pr.K = pr.sc[0].K;
    pr.S_stride = 1;
    for (auto& s : pr.sc) {
        pr.S_stride = std::max(pr.S_stride, s.S);
        if (s.n_bins != pr.n_bins || s.K != pr.K) pr.same_layout = false;
    }
    const int64_t n = pulses->n_pulses;
    if (pulses->n_segments > 0) {
        if (!pulses->segment_offsets || !pulses->segment_scanner)
            return fail(VLS_ERR_INVALID_ARG, "segments need host segment_offsets and segment_scanner");
        if (!pr.same_layout)
            return fail(VLS_ERR_INVALID_ARG, "scanners of one batch must share n_bins and max_returns");
        const int ns = pulses->n_segments;
        pr.off.assign(pulses->segment_offsets, pulses->segment_offsets + ns + 1);
        pr.seg_sc.assign(pulses->segment_scanner, pulses->segment_scanner + ns);
        if (pr.off[0] != 0 || pr.off[ns] != n) return fail(VLS_ERR_INVALID_ARG, "segment offsets must run from 0 to n_pulses");
        for (int s = 0; s < ns; ++s) {
            if (pr.off[s + 1] < pr.off[s]) return fail(VLS_ERR_INVALID_ARG, "segment offsets must not decrease");
            if (pr.seg_sc[s] < 0 || pr.seg_sc[s] >= n_scanners)
                return fail(VLS_ERR_INVALID_ARG, "segment scanner index out of range");
        }
    } else {
        pr.off = {0, n};
        pr.seg_sc = {0};
    }
    return VLS_OK;
}

// allow_tl: the call has a two-level form (vls_trace, vls_simulate).
vls_status check_scene(vls_context ctx, vls_scene scene, const Prepared& pr, bool allow_tl = false)
{
    if (!scene) return fail(VLS_ERR_INVALID_ARG, "scene is NULL");
    if (scene->ctx != ctx) return fail(VLS_ERR_INVALID_ARG, "scene belongs to another context");
    if (scene->tl) {
        if (!allow_tl) return fail(VLS_ERR_UNSUPPORTED, "a two-level scene is traced by vls_trace and vls_simulate only");
        return VLS_OK;
    }
    if (scene->vox.n_vox > 0)
        for (const auto& s : pr.sc)
            if (!(s.vox_c < INFINITY))
                return fail(VLS_ERR_INVALID_ARG, "a scene with voxels needs scanners of divergence > 0 (Eq. 7)");
    int limit = ctx->cfg.stack_lds + kMaxSpill - 1;
    if (scene->stats.max_depth > limit) {
        char b[128];
        snprintf(b, sizeof b, "scene depth %d exceeds the traversal stack (%d)", scene->stats.max_depth, limit);
        return fail(VLS_ERR_UNSUPPORTED, b);
    }
    // the cone pass pushes up to three entries per four-wide level
    const int cone_ring = ctx->cfg.cover_off ? kConeRing : kConeRingCover;
    if (ctx->cfg.cone && 3 * ((scene->stats.max_depth + 1) / 2) > cone_ring + kMaxSpill - 1) {
        char b[128];
        snprintf(b, sizeof b, "scene depth %d exceeds the cone-pass stack; use cone = 0", scene->stats.max_depth);
        return fail(VLS_ERR_UNSUPPORTED, b);
    }
    return VLS_OK;
}

OutDev out_dev(const vls_outputs* o, int stride)
{
    OutDev d;
    memset(&d, 0, sizeof d);
    d.sub_tri = o->subray_tri;
    d.sub_range = o->subray_range;
    d.sub_cos = o->subray_cos;
    d.sub_power = o->subray_power;
    d.sub_stride = stride;
    d.wf = o->waveform;
    d.t0 = o->window_t0_ns;
    d.n_ret = o->n_returns;
    d.ret_range = o->ret_range;
    d.ret_amp = o->ret_amplitude;
    d.ret_tri = o->ret_tri;
    d.ret_bin = o->ret_bin;
    return d;
}

vls_status check_outputs(const vls_outputs* o)
{
    if (!o) return fail(VLS_ERR_INVALID_ARG, "outputs are NULL");
    if (!aligned(o->subray_tri, 4) || !aligned(o->subray_range, 8) || !aligned(o->subray_cos, 4) ||
        !aligned(o->subray_power, 4) || !aligned(o->waveform, 4) || !aligned(o->window_t0_ns, 8) ||
        !aligned(o->n_returns, 4) || !aligned(o->ret_range, 4) || !aligned(o->ret_amplitude, 4) ||
        !aligned(o->ret_tri, 4) || !aligned(o->ret_bin, 4))
        return fail(VLS_ERR_INVALID_ARG, "misaligned output array");
    return VLS_OK;
}

PulsesDev pulses_dev(const vls_pulse_batch* p)
{
    PulsesDev d;
    d.origins = p->origins;
    d.dirs = p->directions;
    d.t0_in = p->window_t0_ns;
    d.n = p->n_pulses;
    d.basis = nullptr;
    d.cand = nullptr;
    d.cand_long = nullptr;
    return d;
}

// Upload (or reuse) the device tables of a segmented batch.
vls_status batch_tables(vls_context ctx, const Prepared& pr, vls_context_s::Batch*& out)
{
    const int ns = (int)pr.seg_sc.size();
    std::vector<long long> tile_off(ns + 1), pulse_off(ns), pulse_end(ns);
    std::vector<int> seg(ns);
    tile_off[0] = 0;
    for (int s = 0; s < ns; ++s) {
        const ScannerDev& sc = pr.sc[pr.seg_sc[s]];
        long long np = pr.off[s + 1] - pr.off[s];
        tile_off[s + 1] = tile_off[s] + (np + sc.P_w - 1) / sc.P_w;
        pulse_off[s] = pr.off[s];
        pulse_end[s] = pr.off[s + 1];
        seg[s] = pr.seg_sc[s];
    }
    // the same segments grouped by scanner (in segment order within a scanner)
    // with their own tile numbering, for one launch per scanner
    const int nsc = (int)pr.sc.size();
    std::vector<long long> g_tile(ns), g_po(ns), g_pe(ns);
    std::vector<int> g_first(nsc + 1, 0);
    std::vector<long long> g_t0(nsc + 1, 0);
    {
        int k = 0;
        long long t = 0;
        for (int c = 0; c < nsc; ++c) {
            g_first[c] = k;
            g_t0[c] = t;
            for (int s = 0; s < ns; ++s) {
                if (pr.seg_sc[s] != c) continue;
                g_tile[k] = t;
                g_po[k] = pulse_off[s];
                g_pe[k] = pulse_end[s];
                t += tile_off[s + 1] - tile_off[s];
                ++k;
            }
        }
        g_first[nsc] = k;
        g_t0[nsc] = t;
    }
    // layout: tile_off | pulse_off | pulse_end | seg | scanners | counter | grouped tile_off | pulse_off | pulse_end
    size_t o_tile = 0, o_po = o_tile + 8 * (ns + 1), o_pe = o_po + 8 * ns, o_seg = o_pe + 8 * ns;
    size_t o_sc = (o_seg + 4 * ns + 63) / 64 * 64, o_ctr = o_sc + sizeof(ScannerDev) * pr.sc.size();
    size_t o_gt = o_ctr + 64, o_gpo = o_gt + 8 * ns, o_gpe = o_gpo + 8 * ns;
    size_t bytes = o_gpe + 8 * ns;
    std::vector<unsigned char> blob(bytes, 0);
    memcpy(&blob[o_tile], tile_off.data(), 8 * (ns + 1));
    memcpy(&blob[o_po], pulse_off.data(), 8 * ns);
    memcpy(&blob[o_pe], pulse_end.data(), 8 * ns);
    memcpy(&blob[o_seg], seg.data(), 4 * ns);
    memcpy(&blob[o_sc], pr.sc.data(), sizeof(ScannerDev) * pr.sc.size());
    memcpy(&blob[o_gt], g_tile.data(), 8 * ns);
    memcpy(&blob[o_gpo], g_po.data(), 8 * ns);
    memcpy(&blob[o_gpe], g_pe.data(), 8 * ns);
    for (auto& b : ctx->batches)
        if (b.key == blob) {
            out = &b;
            return VLS_OK;
        }
    vls_context_s::Batch b;
    VLS_HIP(hipMalloc(&b.dev, bytes), "batch table alloc");
    hipError_t e = hipMemcpy(b.dev, blob.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b.dev);
        return hip_fail(e, "batch table upload");
    }
    b.key = std::move(blob);
    b.bd.tile_off = reinterpret_cast<const long long*>(b.dev + o_tile);
    b.bd.pulse_off = reinterpret_cast<const long long*>(b.dev + o_po);
    b.bd.pulse_end = reinterpret_cast<const long long*>(b.dev + o_pe);
    b.bd.seg_scanner = reinterpret_cast<const int*>(b.dev + o_seg);
    b.bd.scanners = reinterpret_cast<const ScannerDev*>(b.dev + o_sc);
    b.bd.counter = reinterpret_cast<unsigned long long*>(b.dev + o_ctr);
    b.bd.n_seg = ns;
    b.bd.n_tiles = tile_off[ns];
    for (int c = 0; c < nsc; ++c) {
        GroupDev g;
        g.tile_off = reinterpret_cast<const long long*>(b.dev + o_gt) + g_first[c];
        g.pulse_off = reinterpret_cast<const long long*>(b.dev + o_gpo) + g_first[c];
        g.pulse_end = reinterpret_cast<const long long*>(b.dev + o_gpe) + g_first[c];
        g.n_seg = g_first[c + 1] - g_first[c];
        g.tile0 = g_t0[c];
        g.tile1 = g_t0[c + 1];
        b.groups.push_back(g);
    }
    b.max_bins = pr.n_bins;
    ctx->batches.push_back(std::move(b));
    out = &ctx->batches.back();
    return VLS_OK;
}

// Grow a workspace block to `need` bytes in stream order: the old block is
// freed after the work already queued on s (its only user) and the new one is
// usable by work queued after this call.
template <class T>
vls_status ws_grow(T*& p, size_t& have, size_t need, hipStream_t s, const char* what)
{
    if (p && need <= have) return VLS_OK;
    if (p) {
        VLS_HIP(hipFreeAsync(p, s), what);
        p = nullptr;
        have = 0;
    }
    void* q = nullptr;
    VLS_HIP(hipMallocAsync(&q, need < 256 ? 256 : need, s), what);
    p = static_cast<T*>(q);
    have = need < 256 ? 256 : need;
    return VLS_OK;
}

// The workspace of stream s (made on first use).
vls_status stream_ws(vls_context ctx, hipStream_t s, vls_context_s::Workspace*& out)
{
    for (auto& w : ctx->workspaces)
        if (w->stream == s) {
            out = w.get();
            return VLS_OK;
        }
    std::unique_ptr<vls_context_s::Workspace> w(new vls_context_s::Workspace());
    w->stream = s;
    vls_status st = ws_grow(w->ctr, w->ctr_bytes, 64, s, "counter workspace");
    if (st != VLS_OK) return st;
    out = w.get();
    ctx->workspaces.push_back(std::move(w));
    return VLS_OK;
}

// Stream s's workspace with room for the cone pass of n pulses (eager calls only:
// a captured graph brings its own).
vls_status cone_workspace(vls_context ctx, long long n, hipStream_t s, vls_context_s::Workspace*& w)
{
    vls_status st = stream_ws(ctx, s, w);
    if (st != VLS_OK) return st;
    if (!ctx->cfg.cone || n <= 0) return VLS_OK;
    st = ws_grow(w->cand, w->cand_bytes, sizeof(int) * cone_ws_ints(n), s, "candidate workspace");
    if (st != VLS_OK) return st;
    return ws_grow(w->longw, w->long_bytes, sizeof(int) * long_ws_ints(n), s, "long candidate workspace");
}

// The ranging error of every segment's returns, once they are found.
hipError_t range_noise_all(const Prepared& pr, const OutDev& od, hipStream_t s)
{
    for (size_t q = 0; q + 1 < pr.off.size(); ++q) {
        hipError_t e = launch_range_noise(pr.sc[pr.seg_sc[q]], od.n_ret, od.ret_range, pr.off[q],
                                          pr.off[q + 1] - pr.off[q], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

double max_tan(const Prepared& pr)
{
    double t = 0.0;
    for (auto& s : pr.sc) t = std::max(t, s.tan_max);
    return t;
}


}  // namespace

// ------------------------------------------------------------------ ABI

extern "C" {

const char* vls_status_string(vls_status s)
{
    switch (s) {
    case VLS_OK: return "ok";
    case VLS_ERR_INVALID_ARG: return "invalid argument";
    case VLS_ERR_OUT_OF_MEMORY: return "out of memory";
    case VLS_ERR_DEVICE: return "device error";
    case VLS_ERR_NOT_BUILT: return "not built";
    case VLS_ERR_UNSUPPORTED: return "unsupported";
    case VLS_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* vls_last_error(void) { return g_err.c_str(); }

int32_t vls_version(void) { return 1; }

vls_status vls_scanner_subrays(const vls_scanner_desc* scanner, int32_t* n_subrays)
{
    if (!scanner || !n_subrays) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    vls_status st = check_scanner(*scanner, 0);
    if (st != VLS_OK) return st;
    std::vector<double> table;
    int S = subray_table(*scanner, table);
    if (S <= 0) return fail(VLS_ERR_UNSUPPORTED, "subray pattern too large");
    *n_subrays = S;
    return VLS_OK;
}

vls_status vls_context_create(int32_t hip_device, vls_context* out)
{
    try {
        if (!out) return fail(VLS_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        int n = 0;
        VLS_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
        if (hip_device < 0 || hip_device >= n) return fail(VLS_ERR_INVALID_ARG, "no such HIP device");
        VLS_HIP(hipSetDevice(hip_device), "hipSetDevice");
        auto* c = new vls_context_s();
        c->device = hip_device;
        // the allocation-free entry point's scratch on this device (its status is
        // kept and reported by that entry point; other calls do not need it)
        c->noalloc_status = noalloc_scratch(hip_device, &c->noalloc_ptr);
        *out = c;
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_context_destroy(vls_context ctx)
{
    if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
    delete ctx;
    return VLS_OK;
}

vls_status vls_set_launch_config(vls_context ctx, const vls_launch_config* cfg)
{
    if (!ctx || !cfg) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    if (cfg->block_waves != 1 && cfg->block_waves != 2 && cfg->block_waves != 4)
        return fail(VLS_ERR_INVALID_ARG, "block_waves must be 1, 2 or 4");
    int r = cfg->stack_lds;
    if (r < 4 || r > kMaxRing || (r & (r - 1)) != 0) return fail(VLS_ERR_INVALID_ARG, "stack_lds must be 4, 8, 16 or 32");
    if (cfg->persistent_blocks < 0) return fail(VLS_ERR_INVALID_ARG, "persistent_blocks must be >= 0");
    if (cfg->pack != 0 && cfg->pack != 1) return fail(VLS_ERR_INVALID_ARG, "pack must be 0 or 1");
    if (cfg->cone != 0 && cfg->cone != 1) return fail(VLS_ERR_INVALID_ARG, "cone must be 0 or 1");
    if (cfg->cover_off != 0 && cfg->cover_off != 1) return fail(VLS_ERR_INVALID_ARG, "cover_off must be 0 or 1");
    if (cfg->grouped != 0 && cfg->grouped != 1) return fail(VLS_ERR_INVALID_ARG, "grouped must be 0 or 1");
    ctx->cfg.block_waves = cfg->block_waves;
    ctx->cfg.stack_lds = r;
    ctx->cfg.persistent_blocks = cfg->persistent_blocks;
    ctx->cfg.pack = cfg->pack;
    ctx->cfg.cone = cfg->cone;
    ctx->cfg.cover_off = cfg->cover_off;
    ctx->cfg.grouped = cfg->grouped;
    return VLS_OK;
}

vls_status vls_get_launch_config(vls_context ctx, vls_launch_config* cfg)
{
    if (!ctx || !cfg) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    cfg->block_waves = ctx->cfg.block_waves;
    cfg->stack_lds = ctx->cfg.stack_lds;
    cfg->persistent_blocks = ctx->cfg.persistent_blocks;
    cfg->pack = ctx->cfg.pack;
    cfg->cone = ctx->cfg.cone;
    cfg->cover_off = ctx->cfg.cover_off;
    cfg->grouped = ctx->cfg.grouped;
    cfg->reserved = 0;
    return VLS_OK;
}

vls_status vls_scene_create(vls_context ctx, const vls_mesh_desc* mesh, void* stream, vls_scene* out)
{
    try {
        if (!ctx || !mesh || !out) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        const int64_t nv = mesh->n_vertices, nt = mesh->n_triangles;
        if (nv < 0 || nt < 0) return fail(VLS_ERR_INVALID_ARG, "negative sizes");
        if (nt > 0x3fffffff) return fail(VLS_ERR_UNSUPPORTED, "more than 2^30 triangles");
        if (nt > 0 && (nv < 1 || !mesh->vertices || !mesh->triangles || !mesh->reflectance))
            return fail(VLS_ERR_INVALID_ARG, "vertices, triangles and reflectance are required");
        if (mesh->memory != VLS_MEM_HOST && mesh->memory != VLS_MEM_DEVICE)
            return fail(VLS_ERR_INVALID_ARG, "memory must be VLS_MEM_HOST or VLS_MEM_DEVICE");
        VLS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        std::unique_ptr<vls_scene_s> sc(new vls_scene_s());
        sc->ctx = ctx;
        BvhBuffers& b = sc->b;
        b.n_tri = nt;
        b.n_vert = nv;
        const int64_t ni = std::max<int64_t>(nt - 1, 1);
        const int64_t nt1 = std::max<int64_t>(nt, 1), nv1 = std::max<int64_t>(nv, 1);
        int64_t bytes = 0;
        auto alloc = [&](void** p, size_t n) -> hipError_t {
            bytes += (int64_t)n;
            return hipMalloc(p, n);
        };
        VLS_HIP(alloc((void**)&b.nodes, 64 * (size_t)ni), "scene alloc");
        VLS_HIP(alloc((void**)&b.nodes4, 128 * (size_t)ni), "scene alloc");
        VLS_HIP(alloc((void**)&b.tris, 48 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.refl, 4 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.verts, 12 * (size_t)nv1), "scene alloc");
        VLS_HIP(alloc((void**)&b.tri_idx, 12 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.leaf_parent, 4 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.node_parent, 4 * (size_t)ni), "scene alloc");
        VLS_HIP(alloc((void**)&b.leaf_tri, 4 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.morton, 8 * (size_t)nt1), "scene alloc");
        VLS_HIP(alloc((void**)&b.node_depth, 4 * (size_t)ni), "scene alloc");
        VLS_HIP(alloc((void**)&b.level_order, 4 * (size_t)ni), "scene alloc");
        VLS_HIP(alloc((void**)&b.bounds, 4 * 32), "scene alloc");
        VLS_HIP(hipMemsetAsync(b.bounds, 0, 4 * 32, s), "scene init");
        if (nt > 0) {
            hipMemcpyKind kind = mesh->memory == VLS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
            VLS_HIP(hipMemcpyAsync(b.verts, mesh->vertices, 12 * (size_t)nv, kind, s), "vertex copy");
            VLS_HIP(hipMemcpyAsync(b.tri_idx, mesh->triangles, 12 * (size_t)nt, kind, s), "triangle copy");
            VLS_HIP(hipMemcpyAsync(b.refl, mesh->reflectance, 4 * (size_t)nt, kind, s), "reflectance copy");
            // indices and coordinates are checked on the device, before the build
            // reads vertices through the indices
            unsigned bad = 0;
            VLS_HIP(mesh_check(b, s, bad), "mesh check");
            if (bad & 1u) return fail(VLS_ERR_INVALID_ARG, "triangle vertex index out of range");
            if (bad & 2u) return fail(VLS_ERR_INVALID_ARG, "non-finite vertex");
            std::string err;
            hipError_t e = bvh_build(b, s, err);
            if (e != hipSuccess) return hip_fail(e, err.c_str());
        }
        VLS_HIP(hipStreamSynchronize(s), "scene build");
        float host_bounds[16];
        VLS_HIP(hipMemcpy(host_bounds, b.bounds, sizeof host_bounds, hipMemcpyDeviceToHost), "scene stats");
        vls_scene_stats& st = sc->stats;
        st.n_vertices = nv;
        st.n_triangles = nt;
        st.n_internal_nodes = nt > 0 ? nt - 1 : 0;
        st.device_bytes = bytes;
        unsigned depth;
        memcpy(&depth, &host_bounds[13], 4);
        st.max_depth = nt > 0 ? (int32_t)depth : 0;
        st.max_supported_depth = ctx->cfg.stack_lds + kMaxSpill - 1;
        for (int a = 0; a < 3; ++a) {
            st.bounds_lo[a] = host_bounds[a];
            st.bounds_hi[a] = host_bounds[3 + a];
        }
        st.box_pad = 0.0f;
        sc->root = nt >= 2 ? 0 : (nt == 1 ? ~0 : -1);
        *out = sc.release();
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

// Checks scene parts and their instances (shared by the expanded and the
// two-level forms): the placed totals, each instance's first placed vertex and
// triangle (instance order), and the instances of each part.
static vls_status check_placement(const vls_mesh_desc* parts, int32_t n_parts, const vls_instance_desc* instances,
                                  int32_t n_instances, int64_t& V, int64_t& T, std::vector<long long>& voff,
                                  std::vector<long long>& toff, std::vector<std::vector<int>>& of_part)
{
    if ((n_parts > 0 && !parts) || (n_instances > 0 && !instances)) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    if (n_parts < 0 || n_instances < 0) return fail(VLS_ERR_INVALID_ARG, "negative counts");
    for (int p = 0; p < n_parts; ++p) {
        const vls_mesh_desc& m = parts[p];
        if (m.n_vertices < 0 || m.n_triangles < 0) return fail(VLS_ERR_INVALID_ARG, "negative part sizes");
        if ((m.n_vertices > 0 && !m.vertices) ||
            (m.n_triangles > 0 && (!m.triangles || !m.reflectance || m.n_vertices < 1)))
            return fail(VLS_ERR_INVALID_ARG, "a part lacks vertices, triangles or reflectance");
        if (m.memory != VLS_MEM_HOST && m.memory != VLS_MEM_DEVICE)
            return fail(VLS_ERR_INVALID_ARG, "memory must be VLS_MEM_HOST or VLS_MEM_DEVICE");
    }
    V = 0;
    T = 0;
    of_part.assign(n_parts, {});
    voff.assign(n_instances, 0);
    toff.assign(n_instances, 0);
    for (int j = 0; j < n_instances; ++j) {
        const vls_instance_desc& d = instances[j];
        if (d.part < 0 || d.part >= n_parts) return fail(VLS_ERR_INVALID_ARG, "instance part index out of range");
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(d.affine[i])) return fail(VLS_ERR_INVALID_ARG, "non-finite instance map");
        of_part[d.part].push_back(j);
        voff[j] = V;
        toff[j] = T;
        V += parts[d.part].n_vertices;
        T += parts[d.part].n_triangles;
        if (T > 0x3fffffff || V > 0x7fffffff) return fail(VLS_ERR_UNSUPPORTED, "more than 2^30 triangles or 2^31 vertices");
    }
    return VLS_OK;
}

vls_status vls_scene_create_instanced(vls_context ctx, const vls_mesh_desc* parts, int32_t n_parts,
                                      const vls_instance_desc* instances, int32_t n_instances, void* stream,
                                      vls_scene* out)
{
    // device buffers of this call, freed on return (after the stream has finished with them)
    struct Temp {
        std::vector<void*> p;
        ~Temp()
        {
            for (void* q : p) (void)hipFree(q);
        }
        hipError_t alloc(void** q, size_t n)
        {
            hipError_t e = hipMalloc(q, n < 4 ? 4 : n);
            if (e == hipSuccess) p.push_back(*q);
            return e;
        }
    } tmp;
    try {
        if (!ctx || !out) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        int64_t V = 0, T = 0;
        std::vector<long long> voff, toff;
        std::vector<std::vector<int>> of_part;
        vls_status cst = check_placement(parts, n_parts, instances, n_instances, V, T, voff, toff, of_part);
        if (cst != VLS_OK) return cst;
        VLS_HIP(hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        float *wv = nullptr, *wr = nullptr;
        int32_t* wt = nullptr;
        unsigned* bad = nullptr;
        VLS_HIP(tmp.alloc((void**)&wv, 12 * (size_t)V), "instance alloc");
        VLS_HIP(tmp.alloc((void**)&wt, 12 * (size_t)T), "instance alloc");
        VLS_HIP(tmp.alloc((void**)&wr, 4 * (size_t)T), "instance alloc");
        VLS_HIP(tmp.alloc((void**)&bad, 4), "instance alloc");
        VLS_HIP(hipMemsetAsync(bad, 0, 4, s), "instance init");
        for (int p = 0; p < n_parts; ++p) {
            const std::vector<int>& js = of_part[p];
            const vls_mesh_desc& m = parts[p];
            if (js.empty() || (m.n_vertices == 0 && m.n_triangles == 0)) continue;
            const float* pv = m.vertices;
            const int32_t* pt = m.triangles;
            const float* pr = m.reflectance;
            if (m.memory == VLS_MEM_HOST) {
                float *dv = nullptr, *dr = nullptr;
                int32_t* dt = nullptr;
                VLS_HIP(tmp.alloc((void**)&dv, 12 * (size_t)m.n_vertices), "part alloc");
                VLS_HIP(tmp.alloc((void**)&dt, 12 * (size_t)m.n_triangles), "part alloc");
                VLS_HIP(tmp.alloc((void**)&dr, 4 * (size_t)m.n_triangles), "part alloc");
                if (m.n_vertices > 0)
                    VLS_HIP(hipMemcpyAsync(dv, pv, 12 * (size_t)m.n_vertices, hipMemcpyHostToDevice, s), "part copy");
                if (m.n_triangles > 0) {
                    VLS_HIP(hipMemcpyAsync(dt, pt, 12 * (size_t)m.n_triangles, hipMemcpyHostToDevice, s), "part copy");
                    VLS_HIP(hipMemcpyAsync(dr, pr, 4 * (size_t)m.n_triangles, hipMemcpyHostToDevice, s), "part copy");
                }
                pv = dv;
                pt = dt;
                pr = dr;
            }
            const size_t k = js.size();
            std::vector<double> aff(12 * k);
            std::vector<long long> off(2 * k);
            for (size_t q = 0; q < k; ++q) {
                memcpy(&aff[12 * q], instances[js[q]].affine, 12 * sizeof(double));
                off[q] = voff[js[q]];
                off[k + q] = toff[js[q]];
            }
            double* daff = nullptr;
            long long* doff = nullptr;
            VLS_HIP(tmp.alloc((void**)&daff, sizeof(double) * aff.size()), "instance table");
            VLS_HIP(tmp.alloc((void**)&doff, sizeof(long long) * off.size()), "instance table");
            VLS_HIP(hipMemcpyAsync(daff, aff.data(), sizeof(double) * aff.size(), hipMemcpyHostToDevice, s),
                    "instance table");
            VLS_HIP(hipMemcpyAsync(doff, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice, s),
                    "instance table");
            // the host tables must outlive the copies
            VLS_HIP(hipStreamSynchronize(s), "instance table");
            VLS_HIP(launch_instances(pv, pt, pr, m.n_vertices, m.n_triangles, daff, doff, doff + k, (long long)k, wv,
                                     wt, wr, bad, s),
                    "instance expansion");
        }
        unsigned hbad = 0;
        VLS_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "instance check");
        VLS_HIP(hipStreamSynchronize(s), "instance expansion");
        if (hbad) return fail(VLS_ERR_INVALID_ARG, "triangle vertex index out of range in a part");
        vls_mesh_desc world{};
        world.vertices = wv;
        world.triangles = wt;
        world.reflectance = wr;
        world.n_vertices = V;
        world.n_triangles = T;
        world.memory = VLS_MEM_DEVICE;
        return vls_scene_create(ctx, &world, stream, out);
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_scene_create_two_level(vls_context ctx, const vls_mesh_desc* parts, int32_t n_parts,
                                      const vls_instance_desc* instances, int32_t n_instances, void* stream,
                                      vls_scene* out)
{
    try {
        if (!ctx || !out) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        int64_t V = 0, T = 0;
        std::vector<long long> voff, toff;
        std::vector<std::vector<int>> of_part;
        vls_status st = check_placement(parts, n_parts, instances, n_instances, V, T, voff, toff, of_part);
        if (st != VLS_OK) return st;
        // each map's inverse (the ray goes into the part's frame)
        std::vector<InstDev> inst(n_instances);
        for (int j = 0; j < n_instances; ++j) {
            const double* m = instances[j].affine;
            const double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9], k = m[10];
            const double A = e * k - f * h, B = f * g - d * k, C = d * h - e * g;
            const double det = a * A + b * B + c * C;
            if (!(std::fabs(det) > 0.0) || !std::isfinite(1.0 / det))
                return fail(VLS_ERR_UNSUPPORTED, "a two-level scene needs invertible instance maps");
            const double r = 1.0 / det;
            const double M[9] = {A * r, (c * h - b * k) * r, (b * f - c * e) * r,
                                 B * r, (a * k - c * g) * r, (c * d - a * f) * r,
                                 C * r, (b * g - a * h) * r, (a * e - b * d) * r};
            InstDev& I = inst[j];
            memset(&I, 0, sizeof I);
            memcpy(I.m, m, sizeof I.m);
            for (int i = 0; i < 3; ++i) {
                I.inv[4 * i] = M[3 * i];
                I.inv[4 * i + 1] = M[3 * i + 1];
                I.inv[4 * i + 2] = M[3 * i + 2];
                I.inv[4 * i + 3] = -(M[3 * i] * m[3] + M[3 * i + 1] * m[7] + M[3 * i + 2] * m[11]);
            }
            I.part = instances[j].part;
            I.tri_base = (int)toff[j];
        }
        hipStream_t s = (hipStream_t)stream;
        std::unique_ptr<vls_scene_s> sc(new vls_scene_s());
        sc->ctx = ctx;
        sc->tl.reset(new TwoLevelHost());
        TwoLevelHost& tl = *sc->tl;
        tl.parts.assign(n_parts, nullptr);
        std::vector<PartDev> pdev(n_parts);
        memset(pdev.data(), 0, sizeof(PartDev) * pdev.size());
        int64_t bytes = 0, internal = 0;
        int part_depth = 0;
        for (int p = 0; p < n_parts; ++p) {
            if (of_part[p].empty() || parts[p].n_triangles == 0) continue;
            vls_scene q = nullptr;
            if ((st = vls_scene_create(ctx, &parts[p], stream, &q)) != VLS_OK) return st;
            tl.parts[p] = q;
            if (q->stats.max_depth > 63) return fail(VLS_ERR_UNSUPPORTED, "a part's tree is deeper than 63");
            PartDev& P = pdev[p];
            P.nodes = q->b.nodes;
            P.nodes4 = q->b.nodes4;
            P.tris = q->b.tris;
            P.refl = q->b.refl;
            P.root = q->root;
            P.n_tri = (int)q->b.n_tri;
            float mag = 0.0f;
            for (int a = 0; a < 3; ++a) mag = std::max(mag, std::max(std::fabs(q->stats.bounds_lo[a]), std::fabs(q->stats.bounds_hi[a])));
            P.mag = mag;
            bytes += q->stats.device_bytes;
            internal += q->stats.n_internal_nodes;
            part_depth = std::max(part_depth, (int)q->stats.max_depth);
        }
        // the instances' boxes in the scene's frame: the part's box corners mapped
        // in FP64, rounded outward to FP32 (each placed vertex rounds inside them),
        // as degenerate triangles (lo, hi, lo) of the top-level tree; instances of
        // empty parts are left out
        std::vector<float> tv;
        std::vector<int32_t> tt;
        std::vector<InstDev> used;
        for (int j = 0; j < n_instances; ++j) {
            const InstDev& I = inst[j];
            if (!tl.parts[I.part]) continue;
            const vls_scene_stats& ps = tl.parts[I.part]->stats;
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int corner = 0; corner < 8; ++corner) {
                const double x = (corner & 1) ? ps.bounds_hi[0] : ps.bounds_lo[0];
                const double y = (corner & 2) ? ps.bounds_hi[1] : ps.bounds_lo[1];
                const double z = (corner & 4) ? ps.bounds_hi[2] : ps.bounds_lo[2];
                for (int i = 0; i < 3; ++i) {
                    const double w = I.m[4 * i] * x + I.m[4 * i + 1] * y + I.m[4 * i + 2] * z + I.m[4 * i + 3];
                    lo[i] = std::min(lo[i], w);
                    hi[i] = std::max(hi[i], w);
                }
            }
            float flo[3], fhi[3];
            double wmax = 0.0;
            for (int i = 0; i < 3; ++i) {
                // one more step outward covers the rounding of the corner arithmetic itself
                flo[i] = std::nextafter((float)lo[i], -INFINITY);
                fhi[i] = std::nextafter((float)hi[i], INFINITY);
                if (!std::isfinite(flo[i]) || !std::isfinite(fhi[i]))
                    return fail(VLS_ERR_INVALID_ARG, "non-finite placed vertex");
                wmax = std::max(wmax, std::max(std::fabs((double)flo[i]), std::fabs((double)fhi[i])));
            }
            // a placed vertex moves by at most |w| 2^-24 per coordinate when rounded;
            // through A^-1 that is at most |A^-1|_F |w| 2^-23 in the part's frame
            double fro = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int c = 0; c < 3; ++c) fro += I.inv[4 * i + c] * I.inv[4 * i + c];
            InstDev u = I;
            u.pad_local = (float)(std::sqrt(fro) * wmax * 1.1920928955078125e-07 * 1.01);
            used.push_back(u);
            const int32_t base = (int32_t)(tv.size() / 3);
            for (const float* q : {flo, fhi, flo}) tv.insert(tv.end(), q, q + 3);
            tt.insert(tt.end(), {base, base + 1, base + 2});
        }
        std::vector<float> trefl(tt.size() / 3, 0.0f);
        vls_mesh_desc top{};
        top.vertices = tv.data();
        top.triangles = tt.data();
        top.reflectance = trefl.data();
        top.n_vertices = (int64_t)(tv.size() / 3);
        top.n_triangles = (int64_t)(tt.size() / 3);
        top.memory = VLS_MEM_HOST;
        vls_scene q = nullptr;
        if ((st = vls_scene_create(ctx, &top, stream, &q)) != VLS_OK) return st;
        tl.top = q;
        if (q->stats.max_depth > 47) return fail(VLS_ERR_UNSUPPORTED, "the instances' tree is deeper than 47");
        VLS_HIP(hipMalloc(&tl.inst, sizeof(InstDev) * std::max<size_t>(used.size(), 1)), "instance table");
        VLS_HIP(hipMalloc(&tl.parts_dev, sizeof(PartDev) * std::max<size_t>(pdev.size(), 1)), "part table");
        if (!used.empty())
            VLS_HIP(hipMemcpy(tl.inst, used.data(), sizeof(InstDev) * used.size(), hipMemcpyHostToDevice), "instance table");
        if (!pdev.empty())
            VLS_HIP(hipMemcpy(tl.parts_dev, pdev.data(), sizeof(PartDev) * pdev.size(), hipMemcpyHostToDevice), "part table");
        TwoLevelDev& d = tl.dev;
        d.nodes = q->b.nodes;
        d.tris = q->b.tris;
        d.inst = tl.inst;
        d.parts = tl.parts_dev;
        d.root = q->root;
        d.n_leaves = (int)q->b.n_tri;
        d.n_inst = (int)used.size();
        float tmag = 0.0f;
        for (int a = 0; a < 3; ++a) tmag = std::max(tmag, std::max(std::fabs(q->stats.bounds_lo[a]), std::fabs(q->stats.bounds_hi[a])));
        d.mag = tmag;
        vls_scene_stats& ss = sc->stats;
        ss.n_vertices = V;
        ss.n_triangles = T;
        ss.n_internal_nodes = internal + q->stats.n_internal_nodes;
        ss.device_bytes = bytes + q->stats.device_bytes + (int64_t)(sizeof(InstDev) * used.size() + sizeof(PartDev) * pdev.size());
        ss.max_depth = q->stats.max_depth + 1 + part_depth;
        ss.max_supported_depth = 47 + 1 + 63;
        for (int a = 0; a < 3; ++a) {
            ss.bounds_lo[a] = q->stats.bounds_lo[a];
            ss.bounds_hi[a] = q->stats.bounds_hi[a];
        }
        VLS_HIP(hipStreamSynchronize(s), "two-level build");
        *out = sc.release();
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_scene_update_vertices(vls_scene scene, const float* vertices_dev, void* stream)
{
    if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "a two-level scene keeps its parts as built");
    if (!scene || (!vertices_dev && scene->b.n_vert > 0)) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    if (!aligned(vertices_dev, 4)) return fail(VLS_ERR_INVALID_ARG, "misaligned vertices");
    hipStream_t s = (hipStream_t)stream;
    if (scene->b.n_vert > 0)
        VLS_HIP(hipMemcpyAsync(scene->b.verts, vertices_dev, 12 * (size_t)scene->b.n_vert, hipMemcpyDeviceToDevice, s),
                "vertex copy");
    VLS_HIP(bvh_update_vertices(scene->b, s), "refit");
    return VLS_OK;
}

vls_status vls_scene_update_reflectance(vls_scene scene, const float* reflectance_dev, void* stream)
{
    if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "a two-level scene keeps its parts as built");
    if (!scene || (!reflectance_dev && scene->b.n_tri > 0)) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    if (scene->b.n_tri > 0)
        VLS_HIP(hipMemcpyAsync(scene->b.refl, reflectance_dev, 4 * (size_t)scene->b.n_tri, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream),
                "reflectance copy");
    return VLS_OK;
}

vls_status vls_scene_set_voxels(vls_scene scene, const vls_voxel_desc* v, void* stream)
{
    try {
        if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "not available for a two-level scene");
        if (!scene || !v) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
        if (scene->vox.n_vox > 0) return fail(VLS_ERR_INVALID_ARG, "the scene already has a voxel grid");
        if (!v->pad || !v->lut) return fail(VLS_ERR_INVALID_ARG, "pad and lut are required");
        if (v->nx < 1 || v->ny < 1 || v->nz < 1) return fail(VLS_ERR_INVALID_ARG, "grid dimensions must be >= 1");
        const int64_t n_vox = (int64_t)v->nx * v->ny * v->nz;
        if (n_vox > (int64_t)0x7fffffff - scene->b.n_tri)
            return fail(VLS_ERR_UNSUPPORTED, "n_triangles + voxels must stay below 2^31");
        if (!(v->voxel_size_m > 0.0) || !std::isfinite(v->voxel_size_m))
            return fail(VLS_ERR_INVALID_ARG, "voxel_size_m must be finite and > 0");
        const int dims[3] = {v->nx, v->ny, v->nz};
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(v->origin[a]) || !std::isfinite(v->origin[a] + v->voxel_size_m * dims[a]))
                return fail(VLS_ERR_INVALID_ARG, "grid corners must be finite");
        if (v->n_lut < 1) return fail(VLS_ERR_INVALID_ARG, "the leaf-angle table needs a row");
        for (int i = 0; i < v->n_lut; ++i) {
            const double x = v->lut[2 * i], g = v->lut[2 * i + 1];
            if (!std::isfinite(x) || !std::isfinite(g) || g < 0.0)
                return fail(VLS_ERR_INVALID_ARG, "table rows must be finite with g >= 0");
            if (i > 0 && !(x > v->lut[2 * i - 2]))
                return fail(VLS_ERR_INVALID_ARG, "table rows must have strictly increasing vertical components");
        }
        for (int64_t i = 0; i < n_vox; ++i)
            if (!(v->pad[i] >= 0.0f) || !std::isfinite(v->pad[i]))
                return fail(VLS_ERR_INVALID_ARG, "plant area density must be finite and >= 0");
        VLS_HIP(hipSetDevice(scene->ctx->device), "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        float* pad = nullptr;
        double* lut = nullptr;
        VLS_HIP(hipMalloc(&pad, sizeof(float) * (size_t)n_vox), "voxel alloc");
        hipError_t e = hipMalloc(&lut, sizeof(double) * 2 * (size_t)v->n_lut);
        if (e == hipSuccess) e = hipMemcpyAsync(pad, v->pad, sizeof(float) * (size_t)n_vox, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lut, v->lut, sizeof(double) * 2 * (size_t)v->n_lut, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(pad);
            (void)hipFree(lut);
            return hip_fail(e, "voxel upload");
        }
        VoxDev& d = scene->vox;
        d.pad = pad;
        d.lut = lut;
        for (int a = 0; a < 3; ++a) d.origin[a] = v->origin[a];
        d.size = v->voxel_size_m;
        d.nx = v->nx;
        d.ny = v->ny;
        d.nz = v->nz;
        d.n_lut = v->n_lut;
        d.seed = v->seed;
        d.n_vox = n_vox;
        scene->stats.device_bytes += (int64_t)(sizeof(float) * n_vox + sizeof(double) * 2 * v->n_lut);
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_scene_set_specular(vls_scene scene, const float* specularity_dev, const float* exponent_dev,
                                  void* stream)
{
    if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "not available for a two-level scene");
    if (!scene) return fail(VLS_ERR_INVALID_ARG, "scene is NULL");
    if (!specularity_dev && !exponent_dev) {
        scene->spec_on = false;
        return VLS_OK;
    }
    if (!specularity_dev || !exponent_dev) return fail(VLS_ERR_INVALID_ARG, "specularity and exponent go together");
    if (!aligned(specularity_dev, 4) || !aligned(exponent_dev, 4)) return fail(VLS_ERR_INVALID_ARG, "misaligned arrays");
    const int64_t nt = scene->b.n_tri;
    hipStream_t s = (hipStream_t)stream;
    if (!scene->spec) {
        VLS_HIP(hipSetDevice(scene->ctx->device), "hipSetDevice");
        VLS_HIP(hipMalloc(&scene->spec, sizeof(float) * 2 * (size_t)std::max<int64_t>(nt, 1)), "specular alloc");
        scene->stats.device_bytes += (int64_t)(sizeof(float) * 2 * nt);
    }
    if (nt > 0) {
        VLS_HIP(hipMemcpyAsync(scene->spec, specularity_dev, 4 * (size_t)nt, hipMemcpyDeviceToDevice, s), "specular copy");
        VLS_HIP(hipMemcpyAsync(scene->spec + nt, exponent_dev, 4 * (size_t)nt, hipMemcpyDeviceToDevice, s),
                "specular copy");
    }
    scene->spec_on = true;
    return VLS_OK;
}

vls_status vls_scene_stats_get(vls_scene scene, vls_scene_stats* out)
{
    if (!scene || !out) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    *out = scene->stats;
    if (!scene->tl) out->max_supported_depth = scene->ctx->cfg.stack_lds + kMaxSpill - 1;
    return VLS_OK;
}

vls_status vls_scene_export(vls_scene scene, float* nodes, int32_t* leaf_tri, uint64_t* morton, int32_t* root)
{
    if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "not available for a two-level scene");
    if (!scene) return fail(VLS_ERR_INVALID_ARG, "scene is NULL");
    VLS_HIP(hipDeviceSynchronize(), "sync");
    const int64_t nt = scene->b.n_tri;
    if (nodes && nt > 1) VLS_HIP(hipMemcpy(nodes, scene->b.nodes, 64 * (size_t)(nt - 1), hipMemcpyDeviceToHost), "export");
    if (leaf_tri && nt > 0) VLS_HIP(hipMemcpy(leaf_tri, scene->b.leaf_tri, 4 * (size_t)nt, hipMemcpyDeviceToHost), "export");
    if (morton && nt > 0) VLS_HIP(hipMemcpy(morton, scene->b.morton, 8 * (size_t)nt, hipMemcpyDeviceToHost), "export");
    if (root) *root = scene->root;
    return VLS_OK;
}

vls_status vls_scene_destroy(vls_scene scene)
{
    if (!scene) return fail(VLS_ERR_INVALID_ARG, "scene is NULL");
    delete scene;
    return VLS_OK;
}

vls_status vls_trace(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                     const vls_pulse_batch* pulses, const vls_outputs* out, void* stream)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
        if (st != VLS_OK) return st;
        if ((st = check_scene(ctx, scene, pr, true)) != VLS_OK) return st;
        if ((st = check_outputs(out)) != VLS_OK) return st;
        if (pulses->n_pulses > 0 && !out->subray_tri) return fail(VLS_ERR_INVALID_ARG, "subray_tri is required");
        OutDev od = out_dev(out, pr.S_stride);
        PulsesDev pd = pulses_dev(pulses);
        if (scene->tl) {
            for (size_t s = 0; s + 1 < pr.off.size(); ++s) {
                hipError_t e = launch_trace2(scene->tl->dev, pr.sc[pr.seg_sc[s]], pd, od, pr.off[s],
                                             pr.off[s + 1] - pr.off[s], (hipStream_t)stream);
                if (e != hipSuccess) return hip_fail(e, "two-level trace launch");
            }
            return VLS_OK;
        }
        vls_context_s::Workspace* ws = nullptr;
        if ((st = cone_workspace(ctx, pulses->n_pulses, (hipStream_t)stream, ws)) != VLS_OK) return st;
        SceneDev sd = scene_dev(scene);
        if (ctx->cfg.cone && pulses->n_pulses > 0) {
            vls_context_s::Batch* bt = nullptr;
            if (pr.seg_sc.size() > 1 && (st = batch_tables(ctx, pr, bt)) != VLS_OK) return st;
            const long long n = pulses->n_pulses;
            int* list = cone_ws_list(ws->cand, n);
            unsigned long long* ctr = cone_ws_ctr(ws->cand, n);
            double* basis = cone_ws_basis(ws->cand, n);
            hipError_t e = launch_cone(sd, max_tan(pr), pd, ws->cand, 0, n, ctx->cfg, nullptr, list, ctr, basis,
                                       (hipStream_t)stream, ws->longw ? kCandFirst : kCandMax, !ctx->cfg.cover_off);
            if (e != hipSuccess) return hip_fail(e, "cone launch");
            if (ws->longw) {
                pd.basis = basis;
                e = launch_cone_long(sd, max_tan(pr), pd, ws->cand, list, ctr, n, ws->longw, ctx->cfg,
                                     (hipStream_t)stream);
                if (e != hipSuccess) return hip_fail(e, "long-list cone launch");
                list = long_ws_list(ws->longw, n);
                ctr = long_ws_ctr(ws->longw, n);
                pd.cand_long = ws->longw;
            }
            e = launch_packets(sd, pr.sc[0], bt ? bt->bd : BatchDev{}, pd, ws->cand, list, ctr, 0,
                               (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "packet launch");
            pd.cand = ws->cand;
            pd.basis = basis;
        }
        for (size_t s = 0; s + 1 < pr.off.size(); ++s) {
            hipError_t e = launch_simulate(sd, pr.sc[pr.seg_sc[s]], pd, od, pr.off[s], pr.off[s + 1] - pr.off[s], 0,
                                           ctx->cfg, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "trace launch");
        }
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

static vls_status wave_common(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                              const vls_pulse_batch* pulses, const vls_outputs* out, void* stream, int mode)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
        if (st != VLS_OK) return st;
        if ((st = check_outputs(out)) != VLS_OK) return st;
        if (pulses->n_pulses > 0) {
            if (mode == 0 && (!out->subray_tri || !out->subray_range || !out->subray_power || !out->waveform))
                return fail(VLS_ERR_INVALID_ARG, "waveform needs subray_tri, subray_range, subray_power and waveform");
            if (mode == 1 && (!out->waveform || !out->window_t0_ns || !out->n_returns || !out->ret_range ||
                              !out->ret_amplitude || !out->ret_bin))
                return fail(VLS_ERR_INVALID_ARG, "returns need waveform, window_t0_ns and the return arrays");
        }
        OutDev od = out_dev(out, pr.S_stride);
        PulsesDev pd = pulses_dev(pulses);
        for (size_t s = 0; s + 1 < pr.off.size(); ++s) {
            hipError_t e = launch_waveform(pr.sc[pr.seg_sc[s]], pd, od, pr.off[s], pr.off[s + 1] - pr.off[s], mode,
                                           ctx->cfg, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "waveform launch");
        }
        if (mode == 1) {
            hipError_t e = range_noise_all(pr, od, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "ranging error launch");
        }
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_waveform(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, void* stream)
{
    return wave_common(ctx, scanners, n_scanners, pulses, out, stream, 0);
}

vls_status vls_returns(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                       const vls_pulse_batch* pulses, const vls_outputs* out, void* stream)
{
    return wave_common(ctx, scanners, n_scanners, pulses, out, stream, 1);
}

// Multicopter table (Sec. 3.2): per waypoint (x, y, z, start time of the leg
// that starts there, its duration, its length, its start yaw, its end yaw).  A
// leg of length L at cruise speed v and acceleration a lasts L / v + v / a when
// it reaches v (two ramps of v / a, L - v^2 / a at v), else 2 sqrt(L / a).  The
// last row repeats the last leg's end yaw (the platform stays there).
static vls_status copter_table(const vls_survey_desc* sv, std::vector<double>& tab)
{
    const int nw = sv->n_waypoints;
    const double v = sv->speed_mps, a = sv->accel_mps2;
    tab.assign(8 * (size_t)nw, 0.0);
    double start = 0.0;
    for (int i = 0; i < nw; ++i) {
        const double* p = sv->waypoints + 3 * i;
        for (int c = 0; c < 3; ++c) {
            if (!std::isfinite(p[c])) return fail(VLS_ERR_INVALID_ARG, "non-finite waypoint");
            tab[8 * i + c] = p[c];
        }
        tab[8 * i + 3] = start;
        if (i + 1 < nw) {
            const double* q = sv->waypoints + 3 * (i + 1);
            const double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
            const double len = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (!(len > 0.0)) return fail(VLS_ERR_INVALID_ARG, "consecutive waypoints coincide");
            const double dur = v * v / a <= len ? len / v + v / a : 2.0 * std::sqrt(len / a);
            double y0, y1;
            if (sv->leg_yaw) {
                y0 = sv->leg_yaw[2 * i];
                y1 = sv->leg_yaw[2 * i + 1];
                if (!std::isfinite(y0) || !std::isfinite(y1)) return fail(VLS_ERR_INVALID_ARG, "non-finite leg yaw");
            } else {
                y0 = y1 = std::atan2(dy, dx);
            }
            tab[8 * i + 4] = dur;
            tab[8 * i + 5] = len;
            tab[8 * i + 6] = y0;
            tab[8 * i + 7] = y1;
            start = start + dur;
            if (!std::isfinite(start)) return fail(VLS_ERR_INVALID_ARG, "survey too long");
        } else if (i > 0) {
            tab[8 * i + 6] = tab[8 * i + 7] = tab[8 * (i - 1) + 7];
        }
    }
    return VLS_OK;
}

// Pieces of a Multicopter path with smooth turns (Sec. 3.2 banked turns, read as
// coordinated turns): each leg's straight part, and at each interior waypoint
// the circular arc of radius v^2 / (g tan b) tangent to both legs; rows of
// kSmoothRow doubles (see vls_internal.h).  total: the path's length.
static vls_status smooth_table(const vls_survey_desc* sv, std::vector<double>& tab, int& n_piece, double& total)
{
    const int nw = sv->n_waypoints;
    const double v = sv->speed_mps, g = 9.80665;
    const double r = v * v / (g * std::tan(sv->bank_angle_rad));
    const double ramp = v * v / (2.0 * sv->accel_mps2);
    std::vector<double> len(nw > 1 ? nw - 1 : 1), s_at(nw, 0.0);
    std::vector<double> dir(3 * (size_t)std::max(nw - 1, 1));
    for (int j = 0; j + 1 < nw; ++j) {
        const double* a = sv->waypoints + 3 * j;
        const double* b = sv->waypoints + 3 * (j + 1);
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(a[c]) || !std::isfinite(b[c])) return fail(VLS_ERR_INVALID_ARG, "non-finite waypoint");
        const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
        len[j] = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(len[j] > 0.0)) return fail(VLS_ERR_INVALID_ARG, "consecutive waypoints coincide");
        dir[3 * j] = dx / len[j];
        dir[3 * j + 1] = dy / len[j];
        dir[3 * j + 2] = dz / len[j];
    }
    std::vector<double> theta(nw, 0.0);
    for (int i = 1; i + 1 < nw; ++i) {
        const double* u = &dir[3 * (i - 1)];
        const double* w = &dir[3 * i];
        double dot = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
        dot = std::min(1.0, std::max(-1.0, dot));
        theta[i] = std::acos(dot);
        if (theta[i] > 179.0 * M_PI / 180.0) return fail(VLS_ERR_INVALID_ARG, "a smooth turn may not exceed 179 degrees");
        s_at[i] = r * std::tan(0.5 * theta[i]);
    }
    tab.clear();
    n_piece = 0;
    total = 0.0;
    for (int j = 0; j + 1 < nw; ++j) {
        const double need = s_at[j] + s_at[j + 1] + (j == 0 ? ramp : 0.0) + (j + 2 == nw ? ramp : 0.0);
        if (!(need <= len[j]))
            return fail(VLS_ERR_INVALID_ARG, "a leg is too short for its turns and ramps (smooth Multicopter)");
        const double* a = sv->waypoints + 3 * j;
        const double* d = &dir[3 * j];
        double row[kSmoothRow] = {0.0};
        row[0] = total;
        row[1] = len[j] - s_at[j] - s_at[j + 1];
        for (int c = 0; c < 3; ++c) {
            row[5 + c] = a[c] + s_at[j] * d[c];
            row[8 + c] = d[c];
        }
        tab.insert(tab.end(), row, row + kSmoothRow);
        ++n_piece;
        total = total + row[1];
        if (j + 2 < nw && theta[j + 1] > 0.0) {
            const double* b = sv->waypoints + 3 * (j + 1);
            const double* w = &dir[3 * (j + 1)];
            const double dot = std::min(1.0, std::max(-1.0, d[0] * w[0] + d[1] * w[1] + d[2] * w[2]));
            double nv[3] = {w[0] - dot * d[0], w[1] - dot * d[1], w[2] - dot * d[2]};
            const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            double arc[kSmoothRow] = {0.0};
            arc[0] = total;
            arc[1] = r * theta[j + 1];
            arc[2] = 1.0;
            arc[3] = r;
            const double turn_z = d[0] * w[1] - d[1] * w[0];
            arc[4] = turn_z > 0.0 ? sv->bank_angle_rad : (turn_z < 0.0 ? -sv->bank_angle_rad : 0.0);
            for (int c = 0; c < 3; ++c) {
                arc[11 + c] = nv[c] / nn;
                arc[8 + c] = d[c];
                arc[5 + c] = b[c] - s_at[j + 1] * d[c] + r * arc[11 + c];
            }
            tab.insert(tab.end(), arc, arc + kSmoothRow);
            ++n_piece;
            total = total + arc[1];
        }
    }
    if (!std::isfinite(total)) return fail(VLS_ERR_INVALID_ARG, "survey too long");
    return VLS_OK;
}

vls_status vls_generate_pulses(vls_context ctx, const vls_survey_desc* sv, int64_t first, int64_t count,
                               double* origins, float* directions, void* stream)
{
    try {
        if (!ctx || !sv) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
        if (count < 0 || first < 0) return fail(VLS_ERR_INVALID_ARG, "negative pulse range");
        if (sv->n_waypoints < 1 || !sv->waypoints) return fail(VLS_ERR_INVALID_ARG, "need at least one waypoint");
        if (sv->deflector < VLS_DEFLECT_POLYGON || sv->deflector > VLS_DEFLECT_FIBRE)
            return fail(VLS_ERR_INVALID_ARG, "unknown deflector");
        if (!(sv->pulse_rate_hz > 0.0) || !std::isfinite(sv->pulse_rate_hz))
            return fail(VLS_ERR_INVALID_ARG, "pulse_rate_hz must be positive");
        if (!(sv->speed_mps >= 0.0) || !std::isfinite(sv->speed_mps) || !std::isfinite(sv->scan_freq_hz) ||
            !std::isfinite(sv->scan_angle_rad) || !std::isfinite(sv->t0_s) || !(sv->platform_noise_m >= 0.0) ||
            !std::isfinite(sv->platform_noise_m))
            return fail(VLS_ERR_INVALID_ARG, "survey parameters must be finite (speed and noise >= 0)");
        if (sv->deflector == VLS_DEFLECT_FIBRE && sv->n_fibres < 2)
            return fail(VLS_ERR_INVALID_ARG, "a fibre array needs at least two fibres");
        if (sv->platform != VLS_PLATFORM_LINEAR && sv->platform != VLS_PLATFORM_MULTICOPTER &&
            sv->platform != VLS_PLATFORM_MULTICOPTER_SMOOTH)
            return fail(VLS_ERR_INVALID_ARG, "unknown platform");
        const bool copter = sv->platform == VLS_PLATFORM_MULTICOPTER;
        const bool smooth = sv->platform == VLS_PLATFORM_MULTICOPTER_SMOOTH;
        if (!copter && sv->leg_yaw)
            return fail(VLS_ERR_INVALID_ARG, "leg_yaw is for the Multicopter platform without smooth turns");
        if ((copter || smooth) && sv->n_waypoints >= 2 &&
            !(sv->speed_mps > 0.0 && sv->accel_mps2 > 0.0 && std::isfinite(sv->accel_mps2)))
            return fail(VLS_ERR_INVALID_ARG, "a moving Multicopter needs speed_mps > 0 and a finite accel_mps2 > 0");
        if (smooth && !(sv->bank_angle_rad > 0.0 && sv->bank_angle_rad < 0.5 * M_PI))
            return fail(VLS_ERR_INVALID_ARG, "smooth turns need a bank_angle_rad in (0, pi/2)");
        if (count == 0) return VLS_OK;
        if (!origins || !directions) return fail(VLS_ERR_INVALID_ARG, "origins and directions are required");
        if (!aligned(origins, 8) || !aligned(directions, 4)) return fail(VLS_ERR_INVALID_ARG, "misaligned output");
        const int nw = sv->n_waypoints;
        std::vector<double> tab;
        int n_piece = 0;
        double path_len = 0.0;
        if (smooth && nw >= 2) {
            vls_status st = smooth_table(sv, tab, n_piece, path_len);
            if (st != VLS_OK) return st;
        } else if (copter) {
            vls_status st = copter_table(sv, tab);
            if (st != VLS_OK) return st;
        } else {
        // per-waypoint table: position, cumulative length, cos and sin of the
        // heading of the leg that starts there (host FP64)
        tab.resize(6 * (size_t)nw);
        double cum = 0.0;
        for (int i = 0; i < nw; ++i) {
            const double* a = sv->waypoints + 3 * i;
            for (int c = 0; c < 3; ++c) {
                if (!std::isfinite(a[c])) return fail(VLS_ERR_INVALID_ARG, "non-finite waypoint");
                tab[6 * i + c] = a[c];
            }
            if (i > 0) {
                const double* p = sv->waypoints + 3 * (i - 1);
                const double dx = a[0] - p[0], dy = a[1] - p[1], dz = a[2] - p[2];
                const double len = std::sqrt(dx * dx + dy * dy + dz * dz);
                if (!(len > 0.0)) return fail(VLS_ERR_INVALID_ARG, "consecutive waypoints coincide");
                cum = cum + len;
            }
            tab[6 * i + 3] = cum;
            double yaw = 0.0;
            if (i + 1 < nw) {
                const double* b = sv->waypoints + 3 * (i + 1);
                yaw = std::atan2(b[1] - a[1], b[0] - a[0]);
            }
            tab[6 * i + 4] = nw >= 2 ? std::cos(yaw) : 1.0;
            tab[6 * i + 5] = nw >= 2 ? std::sin(yaw) : 0.0;
        }
        }
        // the cache key: the table and its layout
        std::vector<double> key = tab;
        key.push_back((double)sv->platform);
        double* dtab = nullptr;
        for (auto& t : ctx->surveys)
            if (t.key == key) dtab = t.dev;
        if (!dtab) {
            vls_context_s::SurveyTab t;
            VLS_HIP(hipMalloc(&t.dev, sizeof(double) * tab.size()), "survey table");
            hipError_t e = hipMemcpy(t.dev, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(t.dev);
                return hip_fail(e, "survey table upload");
            }
            t.key = key;
            dtab = t.dev;
            ctx->surveys.push_back(std::move(t));
        }
        SurveyDev d;
        d.n_wp = nw;
        d.deflector = sv->deflector;
        d.n_fibres = sv->n_fibres;
        d.platform = sv->platform;
        d.accel = sv->accel_mps2;
        d.speed = sv->speed_mps;
        d.prf = sv->pulse_rate_hz;
        d.freq = sv->scan_freq_hz;
        d.angle = sv->scan_angle_rad;
        d.t0 = sv->t0_s;
        d.noise = sv->platform_noise_m;
        d.seed = sv->seed;
        d.n_piece = n_piece;
        d.path_len = path_len;
        d.t_end = smooth && nw >= 2 ? path_len / sv->speed_mps + sv->speed_mps / sv->accel_mps2 : 0.0;
        hipError_t e = launch_generate(d, dtab, first, count, origins, directions, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "pulse generation launch");
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_echo_width(vls_context ctx, const vls_scanner_desc* scanners, int32_t n_scanners,
                          const vls_pulse_batch* pulses, const vls_outputs* out, float* width_ns, void* stream)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
        if (st != VLS_OK) return st;
        if ((st = check_outputs(out)) != VLS_OK) return st;
        const long long n = pulses->n_pulses;
        if (n == 0) return VLS_OK;
        if (!out->waveform || !out->n_returns || !out->ret_bin || !width_ns)
            return fail(VLS_ERR_INVALID_ARG, "echo width needs waveform, n_returns, ret_bin and width_ns");
        if (!aligned(width_ns, 4)) return fail(VLS_ERR_INVALID_ARG, "misaligned width_ns");
        // workspace: one list entry per return slot, then a 64-bit counter
        const long long entries = n * (long long)pr.K;
        vls_context_s::Workspace* ws = nullptr;
        if ((st = stream_ws(ctx, (hipStream_t)stream, ws)) != VLS_OK) return st;
        if ((st = ws_grow(ws->ew, ws->ew_bytes, sizeof(int) * (size_t)(entries + (entries & 1) + 2), (hipStream_t)stream,
                          "echo-width workspace")) != VLS_OK)
            return st;
        unsigned long long* ctr = reinterpret_cast<unsigned long long*>(ws->ew + entries + (entries & 1));
        for (size_t g = 0; g + 1 < pr.off.size(); ++g) {
            const vls_scanner_desc& d = scanners[pr.seg_sc[g]];
            // start width: the pulse's standard deviation (for Eq. 3 that of a
            // Gaussian of the same width parameter), in bins
            const float s0 = (float)(d.pulse_width_ns / (2.0 * std::sqrt(2.0 * std::log(2.0))) / d.bin_ns);
            hipError_t e = launch_echo_width(pr.sc[pr.seg_sc[g]], out->waveform, out->n_returns, out->ret_bin, s0,
                                             pr.off[g], pr.off[g + 1] - pr.off[g], ws->ew, ctr, width_ns,
                                             (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "echo-width launch");
        }
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

// ws: when not null, gets stream s's workspace, grown for the call (eager
// calls; a graph capture passes null and brings its own).
static vls_status simulate_prepare(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners,
                                   int32_t n_scanners, const vls_pulse_batch* pulses, const vls_outputs* out,
                                   Prepared& pr, vls_context_s::Batch*& bt, int& blocks, hipStream_t s,
                                   vls_context_s::Workspace** ws, bool allow_tl = false)
{
    vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
    if (st != VLS_OK) return st;
    if ((st = check_scene(ctx, scene, pr, allow_tl)) != VLS_OK) return st;
    if ((st = check_outputs(out)) != VLS_OK) return st;
    if (pulses->n_pulses > 0 && (!out->n_returns || !out->ret_range || !out->ret_amplitude || !out->ret_bin))
        return fail(VLS_ERR_INVALID_ARG, "simulate needs n_returns, ret_range, ret_amplitude and ret_bin");
    bt = nullptr;
    blocks = 0;
    if (ws && (st = stream_ws(ctx, s, *ws)) != VLS_OK) return st;
    if (scene->tl) return VLS_OK;
    if (ws && (st = cone_workspace(ctx, pulses->n_pulses, s, *ws)) != VLS_OK) return st;
    if (pulses->n_pulses > 0 && pulses->n_segments > 0) {
        if ((st = batch_tables(ctx, pr, bt)) != VLS_OK) return st;
        blocks = ctx->cfg.persistent_blocks > 0 ? ctx->cfg.persistent_blocks
                                                : persistent_occupancy_blocks(pr.n_bins, staged_slots(pr), scene->vox.n_vox > 0, ctx->cfg);
    }
    return VLS_OK;
}

// Timing events: take a pair from the pool (or create one) and record its start.
static hipError_t prof_begin(vls_context ctx, hipStream_t s, std::pair<hipEvent_t, hipEvent_t>& ev)
{
    hipError_t e;
    if (!ctx->prof_pool.empty()) {
        ev = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
    } else {
        if ((e = hipEventCreate(&ev.first)) != hipSuccess) return e;
        if ((e = hipEventCreate(&ev.second)) != hipSuccess) {
            (void)hipEventDestroy(ev.first);
            return e;
        }
    }
    return hipEventRecord(ev.first, s);
}

static hipError_t prof_end(vls_context ctx, hipStream_t s, std::pair<hipEvent_t, hipEvent_t>& ev,
                           std::vector<std::pair<hipEvent_t, hipEvent_t>>& into)
{
    hipError_t e = hipEventRecord(ev.second, s);
    if (e != hipSuccess) {
        ctx->prof_pool.push_back(ev);
        return e;
    }
    into.push_back(ev);
    return hipSuccess;
}

// cand: candidate workspace of at least n_pulses entries (the context's, or a graph's own)
// allow_prof: timing events may be recorded (not for the allocation-free entry
// point, whose caller may forbid creating them)
// cand, ctr: the cone-pass workspace and the batched launch's work counter (a
// stream's workspace, a graph's own, or the allocation-free entry point's array)
// longw: the long-list workspace, or null (overflowed pulses then all take the
// packet walk; the results are the same)
static vls_status simulate_enqueue(vls_context ctx, vls_scene scene, const Prepared& pr, const vls_pulse_batch* pulses,
                                   const vls_outputs* out, vls_context_s::Batch* bt, int blocks, hipStream_t s,
                                   int* cand, unsigned long long* batch_ctr, bool allow_prof = true,
                                   int* longw = nullptr)
{
    if (pulses->n_pulses == 0) return VLS_OK;
    OutDev od = out_dev(out, pr.S_stride);
    PulsesDev pd = pulses_dev(pulses);
    SceneDev sd = scene_dev(scene);
    hipError_t e;
    // timing events only on eager calls (not while a graph is being captured)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (allow_prof && ctx->prof && hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
    const bool prof = allow_prof && ctx->prof && cap == hipStreamCaptureStatusNone;
    std::pair<hipEvent_t, hipEvent_t> ev{};
    BatchDev bd{};
    if (bt) {
        bd = bt->bd;
        bd.counter = batch_ctr;
    }
    if (ctx->cfg.cone) {
        if (prof && (e = prof_begin(ctx, s, ev)) != hipSuccess) return hip_fail(e, "timing event");
        const long long n = pulses->n_pulses;
        int* list = cone_ws_list(cand, n);
        unsigned long long* ctr = cone_ws_ctr(cand, n);
        double* basis = cone_ws_basis(cand, n);
        e = launch_cone(sd, max_tan(pr), pd, cand, 0, n, ctx->cfg, nullptr, list, ctr, basis, s,
                        longw ? kCandFirst : kCandMax, !ctx->cfg.cover_off);
        if (e != hipSuccess) return hip_fail(e, "cone launch");
        if (longw) {
            // pulses whose row overflowed: a second walk into the long rows
            pd.basis = basis;
            e = launch_cone_long(sd, max_tan(pr), pd, cand, list, ctr, n, longw, ctx->cfg, s);
            if (e != hipSuccess) return hip_fail(e, "long-list cone launch");
            list = long_ws_list(longw, n);
            ctr = long_ws_ctr(longw, n);
            pd.cand_long = longw;
        }
        if (prof && (e = prof_end(ctx, s, ev, ctx->prof_cone)) != hipSuccess) return hip_fail(e, "timing event");
        // pulses whose candidate list overflowed: one wavefront walks each pulse's subrays together
        if (prof && (e = prof_begin(ctx, s, ev)) != hipSuccess) return hip_fail(e, "timing event");
        e = launch_packets(sd, pr.sc[0], bd, pd, cand, list, ctr, 0, s);
        if (e != hipSuccess) return hip_fail(e, "packet launch");
        if (prof && (e = prof_end(ctx, s, ev, ctx->prof_packets)) != hipSuccess) return hip_fail(e, "timing event");
        pd.cand = cand;
        pd.basis = basis;
    }
    if (prof && (e = prof_begin(ctx, s, ev)) != hipSuccess) return hip_fail(e, "timing event");
    if (!bt) {
        e = launch_simulate(sd, pr.sc[0], pd, od, 0, pulses->n_pulses, 1, ctx->cfg, s);
    } else if (ctx->cfg.grouped) {
        e = hipSuccess;
        for (size_t c = 0; c < bt->groups.size() && e == hipSuccess; ++c)
            e = launch_grouped(sd, pr.sc[c], bt->groups[c], pd, od, ctx->cfg, s);
    } else {
        e = launch_persistent(sd, bd, pr.n_bins, staged_slots(pr), pd, od, ctx->cfg, blocks, s);
    }
    if (e != hipSuccess) return hip_fail(e, "simulate launch");
    if (prof && (e = prof_end(ctx, s, ev, ctx->prof_fused)) != hipSuccess) return hip_fail(e, "timing event");
    if ((e = range_noise_all(pr, od, s)) != hipSuccess) return hip_fail(e, "ranging error launch");
    return VLS_OK;
}

// A two-level scene: per-subray hits (k_trace2), then the waveform and the
// returns from them; subray arrays, waveform and window origins the caller did
// not ask for live in a context workspace.
static vls_status simulate_two_level(vls_context ctx, vls_scene scene, const Prepared& pr,
                                     const vls_pulse_batch* pulses, const vls_outputs* out, hipStream_t s,
                                     vls_context_s::Workspace* ws)
{
    const long long n = pulses->n_pulses;
    if (n == 0) return VLS_OK;
    OutDev od = out_dev(out, pr.S_stride);
    const size_t ns = (size_t)n * pr.S_stride;
    size_t need = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = need;
        need += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_tri = od.sub_tri ? 0 : carve(4 * ns);
    const size_t o_rng = od.sub_range ? 0 : carve(8 * ns);
    const size_t o_pow = od.sub_power ? 0 : carve(4 * ns);
    const size_t o_wf = od.wf ? 0 : carve(4 * (size_t)n * pr.n_bins);
    const size_t o_t0 = od.t0 ? 0 : carve(8 * (size_t)n);
    if (need > 0) {
        vls_status st = ws_grow(ws->tlw, ws->tlw_bytes, need, s, "two-level workspace");
        if (st != VLS_OK) return st;
    }
    unsigned char* w = ws->tlw;
    if (!od.sub_tri) od.sub_tri = reinterpret_cast<int32_t*>(w + o_tri);
    if (!od.sub_range) od.sub_range = reinterpret_cast<double*>(w + o_rng);
    if (!od.sub_power) od.sub_power = reinterpret_cast<float*>(w + o_pow);
    if (!od.wf) od.wf = reinterpret_cast<float*>(w + o_wf);
    if (!od.t0) od.t0 = reinterpret_cast<double*>(w + o_t0);
    PulsesDev pd = pulses_dev(pulses);
    for (size_t q = 0; q + 1 < pr.off.size(); ++q) {
        const ScannerDev& sc = pr.sc[pr.seg_sc[q]];
        const long long first = pr.off[q], count = pr.off[q + 1] - pr.off[q];
        hipError_t e = launch_trace2(scene->tl->dev, sc, pd, od, first, count, s);
        if (e == hipSuccess) e = launch_waveform(sc, pd, od, first, count, 0, ctx->cfg, s);
        if (e == hipSuccess) e = launch_waveform(sc, pd, od, first, count, 1, ctx->cfg, s);
        if (e == hipSuccess) e = launch_range_noise(sc, od.n_ret, od.ret_range, first, count, s);
        if (e != hipSuccess) return hip_fail(e, "two-level simulate launch");
    }
    return VLS_OK;
}

vls_status vls_simulate(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, void* stream)
{
    try {
        Prepared pr;
        vls_context_s::Batch* bt = nullptr;
        int blocks = 0;
        vls_context_s::Workspace* ws = nullptr;
        const hipStream_t s = (hipStream_t)stream;
        vls_status st = simulate_prepare(ctx, scene, scanners, n_scanners, pulses, out, pr, bt, blocks, s, &ws, true);
        if (st != VLS_OK) return st;
        if (scene->tl) return simulate_two_level(ctx, scene, pr, pulses, out, s, ws);
        return simulate_enqueue(ctx, scene, pr, pulses, out, bt, blocks, s, ws->cand, ws->ctr, true, ws->longw);
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

static_assert(VLS_NOALLOC_MAX_PULSES == kNoAllocMaxPulses, "vls.h and the library agree on the pulse limit");
static_assert(VLS_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "vls.h and the library agree on the scratch size");

vls_status vls_simulate_noalloc(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanner,
                                const vls_pulse_batch* pulses, const vls_outputs* out, void* stream)
{
    try {
        if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
        if (!pulses) return fail(VLS_ERR_INVALID_ARG, "pulse batch is NULL");
        if (pulses->n_segments != 0)
            return fail(VLS_ERR_UNSUPPORTED, "vls_simulate_noalloc takes one scanner and no segments");
        if (pulses->n_pulses > kNoAllocMaxPulses) {
            char b[160];
            snprintf(b, sizeof b, "vls_simulate_noalloc handles at most %lld pulses per call (got %lld)",
                     (long long)kNoAllocMaxPulses, (long long)pulses->n_pulses);
            return fail(VLS_ERR_INVALID_ARG, b);
        }
        if (scene && scene->tl) return fail(VLS_ERR_UNSUPPORTED, "vls_simulate_noalloc does not take two-level scenes");
        Prepared pr;
        std::vector<std::vector<double>> tables;
        vls_status st = prepare(ctx, scanner, 1, pulses, pr, &tables);
        if (st != VLS_OK) return st;
        if ((st = check_scene(ctx, scene, pr)) != VLS_OK) return st;
        if ((st = check_outputs(out)) != VLS_OK) return st;
        if (pulses->n_pulses > 0 && (!out->n_returns || !out->ret_range || !out->ret_amplitude || !out->ret_bin))
            return fail(VLS_ERR_INVALID_ARG, "simulate needs n_returns, ret_range, ret_amplitude and ret_bin");
        if (ctx->noalloc_status != hipSuccess) return hip_fail(ctx->noalloc_status, "scratch address");
        if (pulses->n_pulses == 0) return VLS_OK;
        hipStream_t s = (hipStream_t)stream;
        // scratch: the subray table, then the cone-pass workspace of this call's pulses
        unsigned char* base = static_cast<unsigned char*>(ctx->noalloc_ptr);
        double* pattern = reinterpret_cast<double*>(base);
        int* cand = reinterpret_cast<int*>(base + kNoAllocPatternBytes);
        hipError_t e = launch_store_pattern(tables[0].data(), (int)tables[0].size(), pattern, s);
        if (e != hipSuccess) return hip_fail(e, "subray table store");
        pr.sc[0].pattern = pattern;
        return simulate_enqueue(ctx, scene, pr, pulses, out, nullptr, 0, s, cand, nullptr, false);
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_trace_counts(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                            const vls_pulse_batch* pulses, uint64_t* counts, void* stream)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
        if (st != VLS_OK) return st;
        if ((st = check_scene(ctx, scene, pr)) != VLS_OK) return st;
        if (!counts) return fail(VLS_ERR_INVALID_ARG, "counts is NULL");
        hipStream_t s = (hipStream_t)stream;
        unsigned long long* dc = nullptr;
        VLS_HIP(hipMalloc(&dc, 3 * sizeof(unsigned long long)), "counts alloc");
        hipError_t e = launch_fill_u64(dc, 3, 0ull, s);
        vls_outputs none;
        memset(&none, 0, sizeof none);
        OutDev od = out_dev(&none, pr.S_stride);
        od.counts = dc;
        PulsesDev pd = pulses_dev(pulses);
        SceneDev sd = scene_dev(scene);
        vls_context_s::Workspace* ws = nullptr;
        if ((st = cone_workspace(ctx, pulses->n_pulses, s, ws)) != VLS_OK) {
            (void)hipFree(dc);
            return st;
        }
        if (e == hipSuccess && ctx->cfg.cone && pulses->n_pulses > 0) {
            double* basis = cone_ws_basis(ws->cand, pulses->n_pulses);
            e = launch_cone(sd, max_tan(pr), pd, ws->cand, 0, pulses->n_pulses, ctx->cfg, dc, nullptr, nullptr, basis,
                            s, kCandMax, !ctx->cfg.cover_off);
            pd.cand = ws->cand;
            pd.basis = basis;
        }
        for (size_t g = 0; e == hipSuccess && g + 1 < pr.off.size(); ++g)
            e = launch_simulate(sd, pr.sc[pr.seg_sc[g]], pd, od, pr.off[g], pr.off[g + 1] - pr.off[g], 2, ctx->cfg, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        unsigned long long h[3] = {0, 0, 0};
        if (e == hipSuccess) e = hipMemcpy(h, dc, sizeof h, hipMemcpyDeviceToHost);
        (void)hipFree(dc);
        if (e != hipSuccess) return hip_fail(e, "trace counts");
        for (int i = 0; i < 3; ++i) counts[i] = h[i];
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_waveform_backward(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanner,
                                 const vls_pulse_batch* pulses, const int32_t* subray_tri, const float* grad_waveform,
                                 float* grad_reflectance, float* grad_vertex_z, void* stream)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanner, 1, pulses, pr);
        if (st != VLS_OK) return st;
        if (!scene || scene->ctx != ctx) return fail(VLS_ERR_INVALID_ARG, "scene is NULL or of another context");
        if (scene->tl) return fail(VLS_ERR_UNSUPPORTED, "not available for a two-level scene");
        if (pulses->n_segments > 0) return fail(VLS_ERR_INVALID_ARG, "the adjoint takes one scanner and no segments");
        if (pulses->n_pulses > 0 && (!pulses->window_t0_ns || !subray_tri || !grad_waveform))
            return fail(VLS_ERR_INVALID_ARG, "the adjoint needs window_t0_ns, subray_tri and grad_waveform");
        if (!grad_reflectance && !grad_vertex_z) return fail(VLS_ERR_INVALID_ARG, "no gradient requested");
        if (!aligned(subray_tri, 4) || !aligned(grad_waveform, 4) || !aligned(grad_reflectance, 4) ||
            !aligned(grad_vertex_z, 4))
            return fail(VLS_ERR_INVALID_ARG, "misaligned array");
        const hipStream_t s = (hipStream_t)stream;
        hipError_t e;
        if (ctx->deterministic) {
            vls_context_s::Workspace* ws = nullptr;
            if ((st = stream_ws(ctx, s, ws)) != VLS_OK) return st;
            if (pulses->n_pulses > 0 &&
                (st = ws_grow(ws->adw, ws->adw_bytes, backward_det_bytes(pulses->n_pulses, pr.sc[0].S), s,
                              "adjoint workspace")) != VLS_OK)
                return st;
            e = launch_backward_det(scene_dev(scene), pr.sc[0], pulses_dev(pulses), subray_tri, pr.S_stride,
                                    grad_waveform, grad_reflectance, grad_vertex_z, scene->b.n_vert, ctx->cfg, ws->adw,
                                    s);
        } else {
            e = launch_backward(scene_dev(scene), pr.sc[0], pulses_dev(pulses), subray_tri, pr.S_stride, grad_waveform,
                                grad_reflectance, grad_vertex_z, scene->b.n_vert, ctx->cfg, s);
        }
        return e == hipSuccess ? VLS_OK : hip_fail(e, "backward launch");
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_set_deterministic(vls_context ctx, int32_t on)
{
    if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
    if (on != 0 && on != 1) return fail(VLS_ERR_INVALID_ARG, "on must be 0 or 1");
    ctx->deterministic = on != 0;
    return VLS_OK;
}

vls_status vls_graph_capture(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                             const vls_pulse_batch* pulses, const vls_outputs* out, vls_graph* graph)
{
    try {
        if (!graph) return fail(VLS_ERR_INVALID_ARG, "graph is NULL");
        *graph = nullptr;
        Prepared pr;
        vls_context_s::Batch* bt = nullptr;
        int blocks = 0;
        vls_status st = simulate_prepare(ctx, scene, scanners, n_scanners, pulses, out, pr, bt, blocks, nullptr,
                                         nullptr);
        if (st != VLS_OK) return st;
        std::unique_ptr<vls_graph_s> g(new vls_graph_s());
        g->ctx = ctx;
        // the graph owns its candidate workspace and work counter: graphs and eager
        // calls replayed on other streams must not share them
        if (ctx->cfg.cone && pulses->n_pulses > 0) {
            VLS_HIP(hipMalloc(&g->cand, sizeof(int) * cone_ws_ints(pulses->n_pulses)), "graph workspace");
            VLS_HIP(hipMalloc(&g->longw, sizeof(int) * long_ws_ints(pulses->n_pulses)), "graph workspace");
        }
        if (bt) VLS_HIP(hipMalloc(&g->ctr, 64), "graph counter");
        VLS_HIP(hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking), "capture stream");
        VLS_HIP(hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal), "begin capture");
        st = simulate_enqueue(ctx, scene, pr, pulses, out, bt, blocks, g->cs, g->cand, g->ctr, true, g->longw);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(g->cs, &gr);
        if (st != VLS_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        g->graph = gr;
        VLS_HIP(hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0), "graph instantiate");
        *graph = g.release();
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_graph_launch(vls_graph graph, void* stream)
{
    if (!graph || !graph->exec) return fail(VLS_ERR_INVALID_ARG, "graph is NULL");
    VLS_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream), "graph launch");
    return VLS_OK;
}

vls_status vls_graph_destroy(vls_graph graph)
{
    if (!graph) return fail(VLS_ERR_INVALID_ARG, "graph is NULL");
    delete graph;
    return VLS_OK;
}

static std::string tune_key(vls_scene scene, const Prepared& pr, const vls_pulse_batch* pulses)
{
    int smin = 64, smax = 1;
    for (auto& s : pr.sc) {
        smin = std::min(smin, s.S);
        smax = std::max(smax, s.S);
    }
    int bucket = 0;
    for (int64_t n = pulses->n_pulses; n > 1; n >>= 1) ++bucket;
    char b[200];
    snprintf(b, sizeof b, "tri=%lld|S=%d-%d|bins=%d|pulses=2^%d|segments=%d", (long long)scene->b.n_tri, smin, smax,
             pr.n_bins, bucket, pulses->n_segments > 0 ? pulses->n_segments : 0);
    return b;
}

static bool tune_cache_find(const char* path, const std::string& key, vls_launch_config& c)
{
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    std::string pat = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, pat.c_str())) continue;
        vls_launch_config t{};
        t.grouped = 1;  // the default for entries written before the field existed
        const char* p;
        if ((p = strstr(line, "\"block_waves\": "))) t.block_waves = atoi(p + 15);
        if ((p = strstr(line, "\"stack_lds\": "))) t.stack_lds = atoi(p + 13);
        if ((p = strstr(line, "\"persistent_blocks\": "))) t.persistent_blocks = atoi(p + 21);
        if ((p = strstr(line, "\"pack\": "))) t.pack = atoi(p + 8);
        if ((p = strstr(line, "\"cone\": "))) t.cone = atoi(p + 8);
        if ((p = strstr(line, "\"cover_off\": "))) t.cover_off = atoi(p + 13);
        if ((p = strstr(line, "\"grouped\": "))) t.grouped = atoi(p + 11);
        c = t;
        found = true;
    }
    fclose(f);
    return found;
}

vls_status vls_autotune(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners, int32_t n_scanners,
                        const vls_pulse_batch* pulses, const vls_outputs* out, const char* cache_path, void* stream,
                        vls_tune_result* result)
{
    try {
        if (!result) return fail(VLS_ERR_INVALID_ARG, "result is NULL");
        memset(result, 0, sizeof *result);
        Prepared pr0;
        vls_context_s::Batch* bt = nullptr;
        int blocks = 0;
        hipStream_t s = (hipStream_t)stream;
        vls_context_s::Workspace* ws = nullptr;
        vls_status st = simulate_prepare(ctx, scene, scanners, n_scanners, pulses, out, pr0, bt, blocks, s, &ws);
        if (st != VLS_OK) return st;
        const std::string key = tune_key(scene, pr0, pulses);
        const LaunchCfg entry = ctx->cfg;
        hipEvent_t e0, e1;
        VLS_HIP(hipEventCreate(&e0), "event");
        VLS_HIP(hipEventCreate(&e1), "event");
        auto timed = [&](const LaunchCfg& c, double& ms) -> vls_status {
            ctx->cfg = c;
            Prepared pr;
            vls_context_s::Batch* b2 = nullptr;
            int bl = 0;
            vls_status r = simulate_prepare(ctx, scene, scanners, n_scanners, pulses, out, pr, b2, bl, s, &ws);
            if (r != VLS_OK) return r;
            if ((r = simulate_enqueue(ctx, scene, pr, pulses, out, b2, bl, s, ws->cand, ws->ctr, true, ws->longw)) != VLS_OK) return r;
            // the fastest of three pairs of launches: single timings vary by a few
            // per cent, as much as the configurations differ
            ms = INFINITY;
            for (int g = 0; g < 3; ++g) {
                VLS_HIP(hipEventRecord(e0, s), "event");
                for (int i = 0; i < 2; ++i)
                    if ((r = simulate_enqueue(ctx, scene, pr, pulses, out, b2, bl, s, ws->cand, ws->ctr, true, ws->longw)) != VLS_OK)
                        return r;
                VLS_HIP(hipEventRecord(e1, s), "event");
                VLS_HIP(hipEventSynchronize(e1), "event");
                float f = 0.0f;
                VLS_HIP(hipEventElapsedTime(&f, e0, e1), "event");
                ms = std::min(ms, f / 2.0);
            }
            return VLS_OK;
        };
        vls_launch_config cached{};
        LaunchCfg best = entry;
        double best_ms = 0.0;
        if ((st = timed(entry, best_ms)) != VLS_OK) { ctx->cfg = entry; return st; }
        result->default_ms = best_ms;
        if (tune_cache_find(cache_path, key, cached)) {
            LaunchCfg c;
            c.block_waves = cached.block_waves;
            c.stack_lds = cached.stack_lds;
            c.persistent_blocks = cached.persistent_blocks;
            c.pack = cached.pack;
            c.cone = cached.cone;
            c.cover_off = cached.cover_off;
            c.grouped = cached.grouped;
            double ms = 0.0;
            if ((st = timed(c, ms)) != VLS_OK) { ctx->cfg = entry; return st; }
            best = c;
            best_ms = ms;
            result->from_cache = 1;
        } else {
            int tried = 1;
            const bool seg = pulses->n_segments > 0;
            int auto_blocks = seg ? persistent_occupancy_blocks(pr0.n_bins, staged_slots(pr0), scene->vox.n_vox > 0, entry) : 0;
            for (int dim = 0; dim < 7; ++dim) {
                std::vector<LaunchCfg> cand;
                for (int v = 0; v < 4; ++v) {
                    LaunchCfg c = best;
                    if (dim == 0) { if (v > 2) break; c.block_waves = 1 << v; }
                    if (dim == 1) c.stack_lds = 4 << v;
                    if (dim == 2) { if (v > 1) break; c.pack = v; }
                    if (dim == 3) { if (!seg || v > 2) break; c.persistent_blocks = v == 0 ? 0 : (v == 1 ? auto_blocks / 2 : 2 * auto_blocks); }
                    if (dim == 4) { if (v > 1) break; c.cone = v; }
                    if (dim == 5) { if (v > 1 || !c.cone) break; c.cover_off = v; }
                    if (dim == 6) { if (v > 1 || !seg) break; c.grouped = v; }
                    if (c.stack_lds + kMaxSpill - 1 < scene->stats.max_depth) continue;
                    cand.push_back(c);
                }
                for (auto& c : cand) {
                    if (c.block_waves == best.block_waves && c.stack_lds == best.stack_lds && c.pack == best.pack &&
                        c.persistent_blocks == best.persistent_blocks && c.cone == best.cone &&
                        c.cover_off == best.cover_off && c.grouped == best.grouped)
                        continue;
                    double ms = 0.0;
                    if ((st = timed(c, ms)) != VLS_OK) { ctx->cfg = entry; return st; }
                    ++tried;
                    if (ms < best_ms) { best_ms = ms; best = c; }
                }
            }
            result->n_tried = tried;
            if (cache_path) {
                FILE* f = fopen(cache_path, "a");
                if (f) {
                    fprintf(f, "{\"key\": \"%s\", \"block_waves\": %d, \"stack_lds\": %d, \"persistent_blocks\": %d, \"pack\": %d, \"cone\": %d, \"cover_off\": %d, \"grouped\": %d, \"ms\": %.6f}\n",
                            key.c_str(), best.block_waves, best.stack_lds, best.persistent_blocks, best.pack, best.cone,
                            best.cover_off, best.grouped, best_ms);
                    fclose(f);
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->cfg = best;
        result->best.block_waves = best.block_waves;
        result->best.stack_lds = best.stack_lds;
        result->best.persistent_blocks = best.persistent_blocks;
        result->best.pack = best.pack;
        result->best.cone = best.cone;
        result->best.cover_off = best.cover_off;
        result->best.grouped = best.grouped;
        result->best_ms = best_ms;
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_cone_candidates(vls_context ctx, vls_scene scene, const vls_scanner_desc* scanners,
                               int32_t n_scanners, const vls_pulse_batch* pulses, int32_t* candidates, void* stream)
{
    try {
        Prepared pr;
        vls_status st = prepare(ctx, scanners, n_scanners, pulses, pr);
        if (st != VLS_OK) return st;
        if ((st = check_scene(ctx, scene, pr)) != VLS_OK) return st;
        if (pulses->n_pulses > 0 && !candidates) return fail(VLS_ERR_INVALID_ARG, "candidates is NULL");
        if (!aligned(candidates, 4)) return fail(VLS_ERR_INVALID_ARG, "misaligned candidates");
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = launch_cone(scene_dev(scene), max_tan(pr), pulses_dev(pulses), candidates, 0, pulses->n_pulses,
                                   ctx->cfg, nullptr, nullptr, nullptr, nullptr, s, kCandMax, !ctx->cfg.cover_off);
        if (e != hipSuccess) return hip_fail(e, "cone launch");
        if (pulses->n_pulses > 0) {
            e = launch_leaf_to_orig(scene->b.leaf_tri, candidates, pulses->n_pulses, s);
            if (e != hipSuccess) return hip_fail(e, "candidate ids");
        }
        return VLS_OK;
    } catch (const std::exception& e) {
        return fail(VLS_ERR_INTERNAL, e.what());
    }
}

vls_status vls_synchronize(vls_context ctx, void* stream)
{
    if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
    VLS_HIP(hipStreamSynchronize((hipStream_t)stream), "synchronize");
    VLS_HIP(hipGetLastError(), "device error");
    return VLS_OK;
}

vls_status vls_profile_enable(vls_context ctx, int32_t enable)
{
    if (!ctx) return fail(VLS_ERR_INVALID_ARG, "context is NULL");
    ctx->prof = enable != 0;
    return VLS_OK;
}

vls_status vls_profile_read(vls_context ctx, vls_profile* out)
{
    if (!ctx || !out) return fail(VLS_ERR_INVALID_ARG, "NULL argument");
    VLS_HIP(hipSetDevice(ctx->device), "set device");
    *out = vls_profile{};
    vls_status st = VLS_OK;
    auto drain = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& ms, int64_t& n) {
        for (auto& e : v) {
            float t = 0.0f;
            hipError_t r = hipEventSynchronize(e.second);
            if (r == hipSuccess) r = hipEventElapsedTime(&t, e.first, e.second);
            if (r != hipSuccess && st == VLS_OK) st = hip_fail(r, "timing event");
            ms += t;
            ++n;
            ctx->prof_pool.push_back(e);
        }
        v.clear();
    };
    drain(ctx->prof_cone, out->cone_ms, out->cone_launches);
    drain(ctx->prof_packets, out->packet_ms, out->packet_launches);
    drain(ctx->prof_fused, out->fused_ms, out->fused_launches);
    return st;
}

}  // extern "C"
