/*
 * FP64 CPU oracle for the virtual-laser-scanning hot path of HELIOS++
 * (Winiwarter et al., "Virtual laser scanning with HELIOS++", arXiv 2101.09154).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the GPU library against a plain,
 * obviously correct definition.  It shares no code with the GPU library.
 *
 * What it computes, per pulse (origin O, direction d):
 *   1. the subray pattern of the beam (Sec. 3.4: concentric rings, floor(2*pi*i)
 *      subrays on ring i plus a central subray) with Gaussian beam weights
 *      (Sec. 3.4, Eq. 1; far-field reading of Eq. 2);
 *   2. each subray's closest hit by brute force over every triangle
 *      (Sec. 3.4: a hit ends the subray; Sec. 5.1: minimum-distance
 *      intersection) with the watertight test of Woop, Benthin & Wald (2013)
 *      in FP64, so that no subray slips through a closed surface along a
 *      shared edge;
 *   3. per-subray return power from the laser radar equation (Sec. 5.2, Eq. 7)
 *      with a Lambertian extended-target cross-section;
 *   4. the full waveform: the sum of the subrays' pulse shapes shifted by
 *      their two-way travel times (Sec. 3.4, Eq. 3 or a Gaussian pulse),
 *      sampled at the bin centres of a window that starts t_pre before the
 *      first return;
 *   5. local maxima of the summed waveform as discrete returns (Sec. 3.4);
 *   6. the analytic gradient of a waveform loss with respect to per-triangle
 *      reflectance and vertex heights (hit selection held fixed);
 *   7. optionally, the width of each return: a Gaussian fitted by non-linear
 *      least squares to the waveform around the return (Sec. 3.4; its cost is
 *      discussed in Sec. 3.6);
 *   8. pulses generated from a survey: a LinearPath, Multicopter or static platform (Sec.
 *      3.2) carrying one of the four scan deflectors of Sec. 3.3, with optional
 *      platform position noise from a counter-based SplitMix64;
 *   9. optionally, transmissive voxels (Sec. 3.5.4, Sec. 5.2): a subray crossing
 *      a voxel of plant area density PAD stops in it at a random depth drawn
 *      from the extinction coefficient (Eq. 5 through a leaf-angle table, Eq. 6),
 *      with the echo power of Eq. 7;
 *   9b. optionally, a ranging error on each return's distance (Sec. 3.7);
 *  10. optionally, a Phong-type specular part of each triangle's response
 *      (Sec. 5.1: materials carry reflectance and specularity);
 *  11. scene parts placed by affine maps (Sec. 3.5: a part loaded several
 *      times and moved by transforms; Sec. 5.1: primitives rotate, scale and
 *      translate): each instance's vertices mapped to the scene's frame.
 * Everything is FP64 with no truncation of the pulse support.
 *
 * Readings where the paper is silent or garbled:
 *   - n_subrays that is not 1 + sum floor(2*pi*i): fill rings in order, the
 *     last ring takes the remainder, evenly spaced;
 *   - ring i of N sits at angle (i/N) * kappa * divergence/2 (divergence is
 *     the full 1/e^2 angle); azimuths 2*pi*m/n_i, no per-ring offset;
 *   - Eq. 2, far field: the beam radius at range R is R*tan(divergence/2), so
 *     a subray at angle a has r/w = tan(a)/tan(divergence/2); weights are
 *     normalised to sum 1;
 *   - Eq. 7 with sigma = pi*rho*cos(theta)*R^2*beta^2 gives
 *     P = P0 * w * (eta * D^2 / 4) * rho * cos(theta) / R^2, cos(theta) = |d.n|;
 *   - two-way time tau = 2R/c; the window origin t0 = min tau - t_pre is not
 *     snapped to a bin grid; bin j samples t0 + j*bin;
 *   - a return is a bin j in [1, n-2] with wf[j] > wf[j-1], wf[j] >= wf[j+1]
 *     and wf[j] >= max(thr_abs, thr_rel * max wf); the first K in time order;
 *     its range is (c/2)(t0 + j*bin - s_peak) where s_peak is the pulse's own
 *     peak offset; it is attributed to the subray contributing most at j
 *     (ties: lowest subray index);
 *   - equal hit distances go to the lowest triangle index; edges are
 *     inclusive; only t > 0 counts;
 *   - echo width (the paper names neither the samples nor the solver): see
 *     the comment above orc_echo_width.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_M_PER_NS 0.299792458 /* speed of light, Sec. 3.4: 299,792,458 m/s */
#define ORC_PI 3.14159265358979323846

enum { ORC_PULSE_GAUSSIAN = 0, ORC_PULSE_EQ3 = 1 };

typedef struct {
    double divergence_rad;      /* full angle at the 1/e^2 points */
    double pattern_extent;      /* kappa: outer ring at kappa * divergence / 2 */
    double pulse_width_ns;      /* Gaussian FWHM, or Eq. 3 pulse length (tau = L / 1.75) */
    double bin_ns;
    double window_pre_ns;       /* < 0: automatic (6 sigma for the Gaussian, 0 for Eq. 3) */
    double peak_power_w;
    double receiver_diameter_m;
    double efficiency;
    double min_echo_abs;
    double min_echo_rel;
    int32_t n_subrays;          /* > 0: ring-fill to this count */
    int32_t beam_quality;       /* used when n_subrays == 0: rings 1..quality */
    int32_t pulse_shape;
    int32_t n_bins;
    int32_t max_returns;
    int32_t pad_;
    double range_noise_m;       /* standard deviation of the ranging error (Sec. 3.7); 0: none */
    uint64_t noise_seed;
} orc_scanner;

/* ------------------------------------------------------------------ pattern (Sec. 3.4, Fig. 6) */

static int ring_capacity(int i) { return (int)floor(2.0 * ORC_PI * (double)i); }

/* Number of subrays on each ring; returns the ring count N (0 for a single ray). */
int orc_ring_layout(int n_subrays, int beam_quality, int32_t* ring_count, int max_rings)
{
    int n = 0;
    if (n_subrays <= 0) {
        if (beam_quality < 0) return -1;
        for (int i = 1; i <= beam_quality; ++i) {
            if (n >= max_rings) return -1;
            ring_count[n++] = ring_capacity(i);
        }
        return n;
    }
    int left = n_subrays - 1;
    for (int i = 1; left > 0; ++i) {
        int m = ring_capacity(i);
        if (m > left) m = left;
        if (n >= max_rings) return -1;
        ring_count[n++] = m;
        left -= m;
    }
    return n;
}

int orc_pattern_size(int n_subrays, int beam_quality)
{
    int32_t rc[256];
    int nr = orc_ring_layout(n_subrays, beam_quality, rc, 256);
    if (nr < 0) return -1;
    int s = 1;
    for (int i = 0; i < nr; ++i) s += rc[i];
    return s;
}

/* Subray k: angle from the beam axis alpha[k], azimuth phi[k], weight[k] (sum 1).
 * Order: the central subray, then ring 1, ring 2, ...  Returns S, or -1. */
int orc_pattern(const orc_scanner* sc, double* alpha, double* phi, double* weight, int cap)
{
    int32_t rc[256];
    int nr = orc_ring_layout(sc->n_subrays, sc->beam_quality, rc, 256);
    if (nr < 0) return -1;
    int s = 1;
    for (int i = 0; i < nr; ++i) s += rc[i];
    if (s > cap) return -1;
    double half = 0.5 * sc->divergence_rad;
    double amax = sc->pattern_extent * half;
    int k = 0;
    alpha[k] = 0.0; phi[k] = 0.0; ++k;
    for (int i = 1; i <= nr; ++i) {
        int m = rc[i - 1];
        for (int q = 0; q < m; ++q) {
            alpha[k] = ((double)i / (double)nr) * amax;
            phi[k] = 2.0 * ORC_PI * (double)q / (double)m;
            ++k;
        }
    }
    /* Eq. 1, I = I0 exp(-2 r^2 / w^2), with r/w = tan(alpha)/tan(divergence/2) */
    double th = tan(half), sum = 0.0;
    for (k = 0; k < s; ++k) {
        double x = (th > 0.0) ? tan(alpha[k]) / th : 0.0;
        weight[k] = exp(-2.0 * x * x);
        sum += weight[k];
    }
    for (k = 0; k < s; ++k) weight[k] /= sum;
    return s;
}

/* ------------------------------------------------------------------ subray directions */

/* Orthonormal basis (u, v) perpendicular to unit n: Duff et al. 2017, "Building
 * an orthonormal basis, revisited". */
static void onb(const double n[3], double u[3], double v[3])
{
    double sgn = copysign(1.0, n[2]);
    double a = -1.0 / (sgn + n[2]);
    double b = n[0] * n[1] * a;
    u[0] = 1.0 + sgn * n[0] * n[0] * a; u[1] = sgn * b; u[2] = -sgn * n[0];
    v[0] = b; v[1] = sgn + n[1] * n[1] * a; v[2] = -n[1];
}

/* Direction of one subray: cos(a) d + sin(a) (cos(phi) u + sin(phi) v), d normalised first. */
void orc_subray_direction(const double d_in[3], double alpha, double phi, double out[3])
{
    double len = sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
    double d[3] = { d_in[0] / len, d_in[1] / len, d_in[2] / len };
    double u[3], v[3];
    onb(d, u, v);
    double ca = cos(alpha), sa = sin(alpha), cp = cos(phi), sp = sin(phi);
    for (int i = 0; i < 3; ++i) out[i] = ca * d[i] + sa * (cp * u[i] + sp * v[i]);
}

/* ------------------------------------------------------------------ closest hit (Sec. 3.4, 5.1) */

static void vload(const float* verts, int32_t idx, double out[3])
{
    out[0] = (double)verts[3 * (int64_t)idx + 0];
    out[1] = (double)verts[3 * (int64_t)idx + 1];
    out[2] = (double)verts[3 * (int64_t)idx + 2];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Watertight ray/triangle test of Woop, Benthin & Wald (2013), in FP64,
 * two-sided, inclusive edges.  The ray is sheared so that it runs along +z;
 * the three 2-D edge functions of the projected triangle are then evaluated
 * from the same operands for both triangles that share an edge, so a ray
 * through a shared edge or vertex is never lost between them.  Returns 1 on a
 * hit with t > 0, with the hit point (1-u-v) a + u b + v c. */
int orc_ray_triangle(const double O[3], const double d[3], const double a[3], const double b[3],
                     const double c[3], double* t, double* u, double* v)
{
    int kz = 0;
    if (fabs(d[1]) > fabs(d[kz])) kz = 1;
    if (fabs(d[2]) > fabs(d[kz])) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (d[kz] < 0.0) { int tmp = kx; kx = ky; ky = tmp; }
    if (d[kz] == 0.0) return 0;
    double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
    double A[3] = { a[0] - O[0], a[1] - O[1], a[2] - O[2] };
    double B[3] = { b[0] - O[0], b[1] - O[1], b[2] - O[2] };
    double C[3] = { c[0] - O[0], c[1] - O[1], c[2] - O[2] };
    double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
    double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
    double Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
    double U = Cx * By - Cy * Bx;   /* edge b-c: weight of a */
    double V = Ax * Cy - Ay * Cx;   /* edge c-a: weight of b */
    double W = Bx * Ay - By * Ax;   /* edge a-b: weight of c */
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return 0;
    double det = U + V + W;
    if (det == 0.0) return 0;
    double T = U * (Sz * A[kz]) + V * (Sz * B[kz]) + W * (Sz * C[kz]);
    double tt = T / det;
    if (!(tt > 0.0)) return 0;
    *t = tt; *u = V / det; *v = W / det;
    return 1;
}

/* Closest hit over all triangles; ties on equal t go to the lowest index.  -1 = miss. */
int64_t orc_closest_hit(const double O[3], const double d[3], const float* verts, const int32_t* tris,
                        int64_t n_tri, double* t_out, double* u_out, double* v_out)
{
    int64_t best = -1;
    double bt = INFINITY, bu = 0.0, bv = 0.0;
    for (int64_t i = 0; i < n_tri; ++i) {
        double a[3], b[3], c[3], t, u, v;
        vload(verts, tris[3 * i + 0], a);
        vload(verts, tris[3 * i + 1], b);
        vload(verts, tris[3 * i + 2], c);
        if (orc_ray_triangle(O, d, a, b, c, &t, &u, &v) && t < bt) {
            best = i; bt = t; bu = u; bv = v;
        }
    }
    *t_out = bt; *u_out = bu; *v_out = bv;
    return best;
}

/* ------------------------------------------------------------------ pulse shape (Sec. 3.4, Eq. 3) */

static double gauss_sigma(const orc_scanner* sc) { return sc->pulse_width_ns / (2.0 * sqrt(2.0 * log(2.0))); }
static double eq3_tau(const orc_scanner* sc) { return sc->pulse_width_ns / 1.75; }

/* Outgoing pulse at time offset s (ns): unit-peak Gaussian, or (s/tau)^2 exp(-s/tau). */
double orc_pulse_value(const orc_scanner* sc, double s)
{
    if (sc->pulse_shape == ORC_PULSE_EQ3) {
        double tau = eq3_tau(sc);
        if (s <= 0.0) return 0.0;
        double x = s / tau;
        return x * x * exp(-x);
    }
    double sg = gauss_sigma(sc);
    return exp(-s * s / (2.0 * sg * sg));
}

/* d/ds of the pulse */
double orc_pulse_derivative(const orc_scanner* sc, double s)
{
    if (sc->pulse_shape == ORC_PULSE_EQ3) {
        double tau = eq3_tau(sc);
        if (s <= 0.0) return 0.0;
        double x = s / tau;
        return (2.0 * x - x * x) * exp(-x) / tau;
    }
    double sg = gauss_sigma(sc);
    return -s / (sg * sg) * exp(-s * s / (2.0 * sg * sg));
}

double orc_window_pre(const orc_scanner* sc)
{
    if (sc->window_pre_ns >= 0.0) return sc->window_pre_ns;
    return sc->pulse_shape == ORC_PULSE_EQ3 ? 0.0 : 6.0 * gauss_sigma(sc);
}

double orc_peak_offset(const orc_scanner* sc) { return sc->pulse_shape == ORC_PULSE_EQ3 ? 2.0 * eq3_tau(sc) : 0.0; }

/* Range of a return at bin j of a window starting at t0 (Sec. 3.4: the point's
 * position along the range axis comes from the local maximum): half the
 * two-way time of the bin, less the pulse's own peak offset, times c. */
double orc_echo_range(const orc_scanner* sc, double t0, int j)
{
    double tj = t0 + (double)j * sc->bin_ns;
    return 0.5 * ORC_C_M_PER_NS * (tj - orc_peak_offset(sc));
}

/* ------------------------------------------------------------------ returns (Sec. 3.4) */

int orc_detect_peaks(const double* wf, int n, double thr_abs, double thr_rel, int K, int32_t* bins)
{
    double mx = 0.0;
    for (int j = 0; j < n; ++j) if (wf[j] > mx) mx = wf[j];
    double thr = thr_rel * mx;
    if (thr_abs > thr) thr = thr_abs;
    int cnt = 0;
    for (int j = 1; j + 1 < n && cnt < K; ++j)
        if (wf[j] > wf[j - 1] && wf[j] >= wf[j + 1] && wf[j] >= thr) bins[cnt++] = j;
    return cnt;
}

/* The subray that contributes most to the waveform at time tj (the return's
 * source, Fig. 4 caption: returns are traceable to objects); ties go to the
 * lowest subray index.  -1 if no subray hit. */
int orc_attribute(const orc_scanner* sc, const int32_t* tri, const double* R, const double* P, int S, double tj)
{
    double best = -1.0;
    int bk = -1;
    for (int k = 0; k < S; ++k) {
        if (tri[k] < 0) continue;
        double q = P[k] * orc_pulse_value(sc, tj - 2.0 * R[k] / ORC_C_M_PER_NS);
        if (q > best) { best = q; bk = k; }
    }
    return bk;
}

/* ------------------------------------------------------------------ one pulse */

static double power_const(const orc_scanner* sc)
{
    return sc->peak_power_w * sc->efficiency * sc->receiver_diameter_m * sc->receiver_diameter_m / 4.0;
}

/* Transmissive voxels (Sec. 3.5.4, Sec. 5.2).  Readings taken:
 *   grid     one axis-aligned grid of cubes of side `size` from `origin`,
 *            nx * ny * nz voxels, PAD per voxel (index ix + nx (iy + ny iz));
 *   sigma    Eq. 5's integral is what the leaf-angle table tabulates (Table 2:
 *            hit probability against the beam's horizontal and vertical
 *            components, obtained by numerical integration); a beam's
 *            horizontal component is sqrt(1 - v_z^2), so the table is a function
 *            of |v_z|: sigma = PAD * g(|v_z|), g linear between the table's rows
 *            (sorted by vertical component) and held at its ends;
 *   depth    Eq. 6: s = -ln(u) / sigma with u uniform in (0, 1]: u =
 *            ((x >> 11) + 1) 2^-53 of SplitMix64 output number
 *            (pulse * 64 + subray) * n_voxels + voxel of the sequence seeded with
 *            `seed`, one draw per voxel a subray crosses;
 *   stop     Sec. 5.2: the subray stops in the voxel when s is at most the length
 *            it travels inside the voxel (Sec. 3.5.4 words the comparison the
 *            other way round; Sec. 5.2 and the physics of extinction agree);
 *            sigma = 0 lets it through;
 *   walk     the voxels are visited in order along the subray (Amanatides & Woo
 *            1987) in FP64; the nearest of the first stopping voxel and the
 *            closest triangle is the hit (Sec. 5.1: consecutive intersections
 *            along the ray);
 *   power    Eq. 7 with the proportionality taken as equality:
 *            P = eta * sigma * P0 w D^2 / (4 pi R^4 beta^2), beta the full
 *            divergence, R the hit distance; cos is reported as 1;
 *   id       a voxel hit is reported as triangle id n_tri + voxel index. */
typedef struct {
    double origin[3];
    double size;
    int32_t nx, ny, nz, n_lut;
    const float* pad;        /* [nz][ny][nx] */
    const double* lut;       /* [n_lut][2]: vertical component, g */
    uint64_t seed;
} orc_voxels;

typedef struct {
    const float* verts; const int32_t* tris; const float* refl; int64_t n_tri;
    const orc_scanner* sc; int S; const double* alpha; const double* phi; const double* w;
    const orc_voxels* vox;   /* NULL: no voxels */
    const float* spec_k;     /* per-triangle specularity, or NULL */
    const float* spec_n;     /* per-triangle Phong exponent */
} orc_ctx;

/* Surface response of a triangle seen at incidence cos ct (Sec. 5.1: materials
 * carry reflectance and specularity; the paper gives no formula).  A
 * Phong-type reading for a scanner whose receiver sits at the emitter: the
 * mirror direction of the beam makes the angle 2 theta with the way back, so
 *   f = (1 - ks) cos theta + ks max(cos 2 theta, 0)^n,  cos 2 theta = 2 ct^2 - 1,
 * which is the Lambertian cos theta for ks = 0 and 1 at normal incidence. */
double orc_surface_response(double ct, double ks, double n)
{
    double c2 = 2.0 * ct * ct - 1.0;
    return (1.0 - ks) * ct + ks * (c2 > 0.0 ? pow(c2, n) : 0.0);
}

/* d f / d cos theta */
double orc_surface_response_dcos(double ct, double ks, double n)
{
    double c2 = 2.0 * ct * ct - 1.0;
    return (1.0 - ks) + (c2 > 0.0 && n != 0.0 ? ks * n * pow(c2, n - 1.0) * 4.0 * ct : 0.0);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t c);

double orc_lut_g(const orc_voxels* v, double vz)
{
    double a = fabs(vz);
    const double* t = v->lut;
    int n = v->n_lut;
    if (a <= t[0]) return t[1];
    if (a >= t[2 * (n - 1)]) return t[2 * (n - 1) + 1];
    int i = 0;
    while (i + 2 < n && t[2 * (i + 1)] <= a) ++i;
    double f = (a - t[2 * i]) / (t[2 * (i + 1)] - t[2 * i]);
    return t[2 * i + 1] + f * (t[2 * (i + 1) + 1] - t[2 * i + 1]);
}

/* The first voxel that stops the ray O + t d (d unit) before t_limit: returns
 * its index (or -1) and sets *t_hit and *sigma.  `counter0` = (pulse * 64 +
 * subray) * n_voxels addresses the draws. */
int64_t orc_voxel_hit(const orc_voxels* v, const double O[3], const double d[3], double t_limit,
                      uint64_t counter0, double* t_hit, double* sigma)
{
    const int n[3] = {v->nx, v->ny, v->nz};
    double t_in = 0.0, t_out = t_limit;
    for (int a = 0; a < 3; ++a)  /* a subray that is not finite meets nothing */
        if (!isfinite(O[a]) || !isfinite(d[a])) return -1;
    for (int a = 0; a < 3; ++a) {
        double lo = v->origin[a], hi = v->origin[a] + v->size * (double)n[a];
        if (d[a] == 0.0) {
            if (O[a] < lo || O[a] > hi) return -1;
            continue;
        }
        double t1 = (lo - O[a]) / d[a], t2 = (hi - O[a]) / d[a];
        if (t1 > t2) { double tt = t1; t1 = t2; t2 = tt; }
        if (t1 > t_in) t_in = t1;
        if (t2 < t_out) t_out = t2;
    }
    if (!(t_in < t_out)) return -1;
    int idx[3], step[3];
    double tmax[3], tdel[3];
    for (int a = 0; a < 3; ++a) {
        /* the entry voxel; a point on a boundary belongs to the voxel the ray
         * moves into */
        double pa = O[a] + t_in * d[a];
        double q = (pa - v->origin[a]) / v->size;
        double f = d[a] < 0.0 ? ceil(q) - 1.0 : floor(q);
        int i = (int)f;
        if (f < 0.0) i = 0;
        if (f > (double)(n[a] - 1)) i = n[a] - 1;
        idx[a] = i;
        if (d[a] > 0.0) {
            step[a] = 1;
            tmax[a] = (v->origin[a] + v->size * (double)(i + 1) - O[a]) / d[a];
            tdel[a] = v->size / d[a];
        } else if (d[a] < 0.0) {
            step[a] = -1;
            tmax[a] = (v->origin[a] + v->size * (double)i - O[a]) / d[a];
            tdel[a] = -v->size / d[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdel[a] = INFINITY;
        }
    }
    const double g = orc_lut_g(v, d[2]);
    double t = t_in;
    while (t < t_out) {
        int ax = 0;
        if (tmax[1] < tmax[ax]) ax = 1;
        if (tmax[2] < tmax[ax]) ax = 2;
        double t_exit = tmax[ax] < t_out ? tmax[ax] : t_out;
        if (t_exit < t) t_exit = t;  /* rounding never walks backwards */
        int64_t vi = (int64_t)idx[0] + (int64_t)v->nx * ((int64_t)idx[1] + (int64_t)v->ny * (int64_t)idx[2]);
        double sg = (double)v->pad[vi] * g;
        if (sg > 0.0) {
            double u = (double)((orc_splitmix64(v->seed, counter0 + (uint64_t)vi) >> 11) + 1) *
                       (1.0 / 9007199254740992.0);
            double sd = -log(u) / sg;
            if (sd <= t_exit - t) {
                *t_hit = t + sd;
                *sigma = sg;
                return vi;
            }
        }
        t = t_exit;
        idx[ax] += step[ax];
        if (idx[ax] < 0 || idx[ax] >= n[ax]) break;
        tmax[ax] += tdel[ax];
    }
    return -1;
}

/* Trace and shade the S subrays of one pulse. */
static void trace_pulse(const orc_ctx* c, int64_t pulse, const double O[3], const float d32[3],
                        int32_t* tri, double* R, double* cosang, double* P, double* U, double* V)
{
    double d[3] = { d32[0], d32[1], d32[2] };
    double C = power_const(c->sc);
    for (int k = 0; k < c->S; ++k) {
        double dk[3], t, u, v;
        orc_subray_direction(d, c->alpha[k], c->phi[k], dk);
        int64_t h = orc_closest_hit(O, dk, c->verts, c->tris, c->n_tri, &t, &u, &v);
        if (c->vox) {
            double tv, sg;
            uint64_t c0 = ((uint64_t)pulse * 64 + (uint64_t)k) *
                          (uint64_t)((int64_t)c->vox->nx * c->vox->ny * c->vox->nz);
            int64_t vi = orc_voxel_hit(c->vox, O, dk, h >= 0 ? t : INFINITY, c0, &tv, &sg);
            if (vi >= 0) {
                /* Eq. 7, proportionality taken as equality */
                double beta = c->sc->divergence_rad;
                double Dm = c->sc->receiver_diameter_m;
                tri[k] = (int32_t)(c->n_tri + vi);
                R[k] = tv;
                cosang[k] = 1.0;
                U[k] = V[k] = 0.0;
                P[k] = c->sc->efficiency * sg * c->sc->peak_power_w * c->w[k] * Dm * Dm /
                       (4.0 * ORC_PI * tv * tv * tv * tv * beta * beta);
                continue;
            }
        }
        tri[k] = (int32_t)h;
        if (h < 0) { R[k] = INFINITY; cosang[k] = 0.0; P[k] = 0.0; U[k] = V[k] = 0.0; continue; }
        double a[3], b[3], cc[3], e1[3], e2[3], n[3];
        vload(c->verts, c->tris[3 * h + 0], a);
        vload(c->verts, c->tris[3 * h + 1], b);
        vload(c->verts, c->tris[3 * h + 2], cc);
        for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = cc[i] - a[i]; }
        cross3(e1, e2, n);
        double ct = fabs(dot3(dk, n)) / sqrt(dot3(n, n));
        R[k] = t; cosang[k] = ct; U[k] = u; V[k] = v;
        /* Eq. 7 with a Lambertian extended-target cross-section */
        double f = c->spec_k ? orc_surface_response(ct, c->spec_k[h], c->spec_n[h]) : ct;
        P[k] = C * c->w[k] * (double)c->refl[h] * f / (t * t);
    }
}

/* Waveform + returns for one pulse from its traced subrays. */
/* Ranging error of return r of pulse p (Sec. 3.7: each distance measurement
 * carries a normally distributed error with the scanner's parameters; mean 0
 * and standard deviation sigma here): Box-Muller on the uniforms
 * ((x >> 11) + 1) 2^-53 of SplitMix64 outputs 2 (p K + r) and 2 (p K + r) + 1
 * of the sequence seeded with the scanner's noise seed. */
double orc_range_noise(const orc_scanner* sc, int64_t p, int r)
{
    if (!(sc->range_noise_m > 0.0)) return 0.0;
    uint64_t c = 2 * ((uint64_t)p * (uint64_t)sc->max_returns + (uint64_t)r);
    double u1 = (double)((orc_splitmix64(sc->noise_seed, c) >> 11) + 1) * (1.0 / 9007199254740992.0);
    double u2 = (double)((orc_splitmix64(sc->noise_seed, c + 1) >> 11) + 1) * (1.0 / 9007199254740992.0);
    return sc->range_noise_m * sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
}

static void waveform_pulse(const orc_ctx* c, int64_t pulse, const int32_t* tri, const double* R, const double* P,
                           const double* t0_in, double* wf, double* t0_out, int32_t* n_ret,
                           double* ret_range, double* ret_amp, int32_t* ret_tri, int32_t* ret_bin)
{
    const orc_scanner* sc = c->sc;
    int nb = sc->n_bins, K = sc->max_returns;
    double tmin = INFINITY;
    int any = 0;
    for (int k = 0; k < c->S; ++k)
        if (tri[k] >= 0) { any = 1; double tau = 2.0 * R[k] / ORC_C_M_PER_NS; if (tau < tmin) tmin = tau; }
    double t0 = t0_in ? *t0_in : (any ? tmin - orc_window_pre(sc) : NAN);
    *t0_out = t0;
    for (int j = 0; j < nb; ++j) wf[j] = 0.0;
    for (int r = 0; r < K; ++r) { ret_range[r] = 0.0; ret_amp[r] = 0.0; ret_tri[r] = -1; ret_bin[r] = -1; }
    *n_ret = 0;
    if (!any || isnan(t0)) return;
    for (int j = 0; j < nb; ++j) {
        double tj = t0 + (double)j * sc->bin_ns, acc = 0.0;
        for (int k = 0; k < c->S; ++k)
            if (tri[k] >= 0) acc += P[k] * orc_pulse_value(sc, tj - 2.0 * R[k] / ORC_C_M_PER_NS);
        wf[j] = acc;
    }
    int32_t bins[64];
    int cnt = orc_detect_peaks(wf, nb, sc->min_echo_abs, sc->min_echo_rel, K, bins);
    *n_ret = cnt;
    for (int r = 0; r < cnt; ++r) {
        int j = bins[r];
        double tj = t0 + (double)j * sc->bin_ns;
        int bk = orc_attribute(sc, tri, R, P, c->S, tj);
        ret_bin[r] = j;
        ret_amp[r] = wf[j];
        ret_range[r] = orc_echo_range(sc, t0, j) + orc_range_noise(sc, pulse, r);
        ret_tri[r] = bk >= 0 ? tri[bk] : -1;
    }
}

static int make_ctx(orc_ctx* c, const float* verts, const int32_t* tris, const float* refl, int64_t n_tri,
                    const orc_scanner* sc, double* alpha, double* phi, double* w)
{
    c->verts = verts; c->tris = tris; c->refl = refl; c->n_tri = n_tri; c->sc = sc;
    c->alpha = alpha; c->phi = phi; c->w = w;
    c->vox = NULL;
    c->spec_k = NULL;
    c->spec_n = NULL;
    c->S = orc_pattern(sc, alpha, phi, w, 4096);
    if (c->S <= 0 || sc->n_bins < 3 || sc->max_returns < 1 || sc->max_returns > 64 || !(sc->bin_ns > 0.0)) return -1;
    return 0;
}

/* Full forward over a selection of pulses (sel == NULL: all).  Output q belongs
 * to pulse sel[q].  Per-subray arrays are [n_sel][S]; waveform [n_sel][n_bins];
 * returns [n_sel][K].  t0_in (indexed by pulse, may be NULL) fixes the window
 * origins.  Any per-subray output may be NULL.  Returns S, or -1. */
/* The same with transmissive voxels and specular materials (vox, spec_k and
 * spec_n may be NULL). */
int orc_simulate_ext(const float* verts, int64_t n_vert, const int32_t* tris, const float* refl, int64_t n_tri,
                     const orc_scanner* sc, const double* origins, const float* dirs, int64_t n_pulses,
                     const int64_t* sel, int64_t n_sel, const double* t0_in,
                     int32_t* sub_tri, double* sub_range, double* sub_cos, double* sub_power,
                     double* sub_u, double* sub_v,
                     double* wf, double* t0_out, int32_t* n_ret, double* ret_range, double* ret_amp,
                     int32_t* ret_tri, int32_t* ret_bin, int n_threads, const orc_voxels* vox,
                     const float* spec_k, const float* spec_n)
{
    (void)n_vert;
    double alpha[4096], phi[4096], w[4096];
    orc_ctx c;
    if (make_ctx(&c, verts, tris, refl, n_tri, sc, alpha, phi, w) < 0) return -1;
    c.vox = vox;
    c.spec_k = spec_k;
    c.spec_n = spec_n;
    int S = c.S, nb = sc->n_bins, K = sc->max_returns;
    int64_t n = sel ? n_sel : n_pulses;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        int32_t* tri = (int32_t*)malloc(sizeof(int32_t) * S);
        double* R = (double*)malloc(sizeof(double) * S * 5);
        double *cs = R + S, *P = R + 2 * S, *U = R + 3 * S, *V = R + 4 * S;
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; ++q) {
            int64_t p = sel ? sel[q] : q;
            trace_pulse(&c, p, origins + 3 * p, dirs + 3 * p, tri, R, cs, P, U, V);
            for (int k = 0; k < S; ++k) {
                if (sub_tri) sub_tri[q * S + k] = tri[k];
                if (sub_range) sub_range[q * S + k] = R[k];
                if (sub_cos) sub_cos[q * S + k] = cs[k];
                if (sub_power) sub_power[q * S + k] = P[k];
                if (sub_u) sub_u[q * S + k] = U[k];
                if (sub_v) sub_v[q * S + k] = V[k];
            }
            if (wf) {
                waveform_pulse(&c, p, tri, R, P, t0_in ? t0_in + p : NULL, wf + q * nb, t0_out + q, n_ret + q,
                               ret_range + q * K, ret_amp + q * K, ret_tri + q * K, ret_bin + q * K);
            }
        }
        free(tri);
        free(R);
    }
    return S;
}

int orc_simulate(const float* verts, int64_t n_vert, const int32_t* tris, const float* refl, int64_t n_tri,
                 const orc_scanner* sc, const double* origins, const float* dirs, int64_t n_pulses,
                 const int64_t* sel, int64_t n_sel, const double* t0_in,
                 int32_t* sub_tri, double* sub_range, double* sub_cos, double* sub_power,
                 double* sub_u, double* sub_v,
                 double* wf, double* t0_out, int32_t* n_ret, double* ret_range, double* ret_amp,
                 int32_t* ret_tri, int32_t* ret_bin, int n_threads)
{
    return orc_simulate_ext(verts, n_vert, tris, refl, n_tri, sc, origins, dirs, n_pulses, sel, n_sel, t0_in, sub_tri,
                            sub_range, sub_cos, sub_power, sub_u, sub_v, wf, t0_out, n_ret, ret_range, ret_amp,
                            ret_tri, ret_bin, n_threads, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------ gradient */

/* Gradient of L(wf) for wf computed with fixed window origins t0[p], given
 * G = dL/dwf [n_pulses][n_bins], with respect to reflectance [n_tri] and
 * vertex heights z [n_vert].  Hit selection is recomputed by brute force at
 * the current geometry and then held fixed.  Chain: P = C w rho cos/R^2,
 * tau = 2R/c, R = n.(a-O)/(n.d) so dR/dv_i = b_i n/(n.d) (b_i = barycentric
 * weight of vertex i at the hit), cos = |n.d|/|n|.  Accumulated per thread in
 * thread order (deterministic for a fixed thread count). */
/* The same with transmissive voxels and specular materials (vox, spec_k and
 * spec_n may be NULL): a subray that a voxel stops carries no triangle and so
 * adds nothing to either gradient; the surface response f replaces cos theta
 * in P and df/dcos carries the incidence derivative. */
int orc_gradient_ext(const float* verts, int64_t n_vert, const int32_t* tris, const float* refl, int64_t n_tri,
                     const orc_scanner* sc, const double* origins, const float* dirs, int64_t n_pulses,
                     const double* t0, const double* grad_wf, double* grad_refl, double* grad_z, int n_threads,
                     const orc_voxels* vox, const float* spec_k, const float* spec_n)
{
    double alpha[4096], phi[4096], w[4096];
    orc_ctx c;
    if (make_ctx(&c, verts, tris, refl, n_tri, sc, alpha, phi, w) < 0) return -1;
    c.vox = vox;
    c.spec_k = spec_k;
    c.spec_n = spec_n;
    int S = c.S, nb = sc->n_bins;
    double C = power_const(sc);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
    int nth = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
    int nth = 1;
#endif
    double* part = (double*)calloc((size_t)nth * (size_t)(n_tri + n_vert), sizeof(double));
    if (!part) return -1;
#pragma omp parallel num_threads(nth)
    {
#ifdef _OPENMP
        int me = omp_get_thread_num();
#else
        int me = 0;
#endif
        double* gr = part + (size_t)me * (size_t)(n_tri + n_vert);
        double* gz = gr + n_tri;
        int32_t* tri = (int32_t*)malloc(sizeof(int32_t) * S);
        double* R = (double*)malloc(sizeof(double) * S * 5);
        double *cs = R + S, *P = R + 2 * S, *U = R + 3 * S, *V = R + 4 * S;
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < n_pulses; ++p) {
            if (isnan(t0[p])) continue;
            trace_pulse(&c, p, origins + 3 * p, dirs + 3 * p, tri, R, cs, P, U, V);
            double dp[3] = { dirs[3 * p], dirs[3 * p + 1], dirs[3 * p + 2] };
            const double* G = grad_wf + p * nb;
            for (int k = 0; k < S; ++k) {
                int32_t h = tri[k];
                if (h < 0 || h >= n_tri) continue;
                double tau = 2.0 * R[k] / ORC_C_M_PER_NS, gP = 0.0, gD = 0.0;
                for (int j = 0; j < nb; ++j) {
                    double s = t0[p] + (double)j * sc->bin_ns - tau;
                    gP += G[j] * orc_pulse_value(sc, s);
                    gD += G[j] * orc_pulse_derivative(sc, s);
                }
                double gtau = -P[k] * gD;                   /* d wf_j / d tau = -P p'(s) */
                double gR = gtau * 2.0 / ORC_C_M_PER_NS - gP * 2.0 * P[k] / R[k];
                double base = C * w[k] / (R[k] * R[k]);
                double f = spec_k ? orc_surface_response(cs[k], spec_k[h], spec_n[h]) : cs[k];
                double df = spec_k ? orc_surface_response_dcos(cs[k], spec_k[h], spec_n[h]) : 1.0;
                double gcos = gP * base * (double)refl[h] * df;
                gr[h] += gP * base * f;
                double dk[3], a[3], b[3], cc[3], e1[3], e2[3], n[3];
                orc_subray_direction(dp, alpha[k], phi[k], dk);
                vload(verts, tris[3 * h + 0], a);
                vload(verts, tris[3 * h + 1], b);
                vload(verts, tris[3 * h + 2], cc);
                for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = cc[i] - a[i]; }
                cross3(e1, e2, n);
                double nd = dot3(n, dk), nn = sqrt(dot3(n, n));
                double bary[3] = { 1.0 - U[k] - V[k], U[k], V[k] };
                for (int i = 0; i < 3; ++i) gz[tris[3 * h + i]] += gR * bary[i] * n[2] / nd;
                /* cos = sgn(nd) nd/|n|: d cos/d n = sgn (d/|n| - nd n/|n|^3) */
                double sg = nd >= 0.0 ? 1.0 : -1.0, gn[3];
                for (int i = 0; i < 3; ++i) gn[i] = gcos * sg * (dk[i] / nn - nd * n[i] / (nn * nn * nn));
                double d12[3] = { e1[0] - e2[0], e1[1] - e2[1], e1[2] - e2[2] }, r0[3], r1[3], r2[3];
                cross3(d12, gn, r0);   /* dn = dv0 x (e1 - e2) */
                cross3(e2, gn, r1);    /* dn = dv1 x e2        */
                cross3(gn, e1, r2);    /* dn = e1 x dv2        */
                gz[tris[3 * h + 0]] += r0[2];
                gz[tris[3 * h + 1]] += r1[2];
                gz[tris[3 * h + 2]] += r2[2];
            }
        }
        free(tri);
        free(R);
    }
    for (int64_t i = 0; i < n_tri; ++i) grad_refl[i] = 0.0;
    for (int64_t i = 0; i < n_vert; ++i) grad_z[i] = 0.0;
    for (int t = 0; t < nth; ++t) {
        double* gr = part + (size_t)t * (size_t)(n_tri + n_vert);
        for (int64_t i = 0; i < n_tri; ++i) grad_refl[i] += gr[i];
        for (int64_t i = 0; i < n_vert; ++i) grad_z[i] += gr[n_tri + i];
    }
    free(part);
    return S;
}

int orc_gradient(const float* verts, int64_t n_vert, const int32_t* tris, const float* refl, int64_t n_tri,
                 const orc_scanner* sc, const double* origins, const float* dirs, int64_t n_pulses,
                 const double* t0, const double* grad_wf, double* grad_refl, double* grad_z, int n_threads)
{
    return orc_gradient_ext(verts, n_vert, tris, refl, n_tri, sc, origins, dirs, n_pulses, t0, grad_wf, grad_refl,
                            grad_z, n_threads, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------ echo width (Sec. 3.4, optional) */

/* The paper fits a Gaussian to the waveform of each return by non-linear least
 * squares and reports its standard deviation as the echo width; the return's
 * position stays the local maximum.  Readings taken where it says no more:
 *   samples  the return's lobe: from the return bin j outward while the
 *            waveform keeps falling strictly and stays at or above 2^-10 of
 *            wf[j] (the tails below carry next to nothing), at most ORC_EW_HALF
 *            bins to each side and within the waveform;
 *   model    g(x) = A exp(-(x - mu)^2 / (2 s^2)), x = bin index - j;
 *   start    the Gaussian through bins j-1, j, j+1 (a parabola through the
 *            logarithms) when those three lie in the lobe, are positive and
 *            curve downward; otherwise A = wf[j], mu = 0, s = s0 (the pulse's
 *            own standard deviation in bins);
 *   solver   Levenberg-Marquardt: solve (J'J + lambda diag(J'J)) delta = J'r
 *            for the residuals r = wf - g; accept p + delta if its centre lies
 *            within the lobe's length of j, its |s| is at most twice the number
 *            of lobe bins, and it lowers the sum of squares (lambda / 10); else
 *            keep p (lambda * 10); lambda starts at 1e-3; exactly ORC_EW_ITERS
 *            iterations;
 *   result   |s| times the bin width, in ns; NaN for a lobe of fewer than
 *            three bins, a singular system at the start, or a fit that ends
 *            with A <= 0 or a non-finite s. */
#define ORC_EW_HALF 31
#define ORC_EW_ITERS 12

/* Sum of squared residuals, and J'J (upper triangle: 00 01 02 11 12 22) and
 * J'r at p = (A, mu, s) over the samples (x[i], y[i]). */
static double ew_normal(const double* x, const double* y, int m, const double p[3], double H[6], double g[3])
{
    double c = 0.0;
    for (int q = 0; q < 6; ++q) H[q] = 0.0;
    for (int q = 0; q < 3; ++q) g[q] = 0.0;
    for (int i = 0; i < m; ++i) {
        double d = x[i] - p[1];
        double e = exp(-d * d / (2.0 * p[2] * p[2]));
        double r = y[i] - p[0] * e;
        double J[3] = {e, p[0] * e * d / (p[2] * p[2]), p[0] * e * d * d / (p[2] * p[2] * p[2])};
        c += r * r;
        H[0] += J[0] * J[0];
        H[1] += J[0] * J[1];
        H[2] += J[0] * J[2];
        H[3] += J[1] * J[1];
        H[4] += J[1] * J[2];
        H[5] += J[2] * J[2];
        for (int q = 0; q < 3; ++q) g[q] += J[q] * r;
    }
    return c;
}

static double ew_cost(const double* x, const double* y, int m, const double p[3])
{
    double c = 0.0;
    for (int i = 0; i < m; ++i) {
        double d = x[i] - p[1];
        double r = y[i] - p[0] * exp(-d * d / (2.0 * p[2] * p[2]));
        c += r * r;
    }
    return c;
}

/* Solves the symmetric 3x3 system M delta = g (M from its upper triangle) by
 * Cramer's rule; 0 if it is singular. */
static int ew_solve(const double M[6], const double g[3], double delta[3])
{
    double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5];
    double det = a * (d * f - e * e) - b * (b * f - e * c) + c * (b * e - d * c);
    if (!(det != 0.0) || !isfinite(det)) return 0;
    delta[0] = (g[0] * (d * f - e * e) - b * (g[1] * f - e * g[2]) + c * (g[1] * e - d * g[2])) / det;
    delta[1] = (a * (g[1] * f - e * g[2]) - g[0] * (b * f - e * c) + c * (b * g[2] - g[1] * c)) / det;
    delta[2] = (a * (d * g[2] - g[1] * e) - b * (b * g[2] - g[1] * c) + g[0] * (b * e - d * c)) / det;
    return 1;
}

/* Echo width of the return at bin j of the waveform wf[0..n-1]; s0: the start
 * width in bins; returns the width in bins (NaN: no fit).  p_out (optional)
 * receives the fitted (A, mu, s). */
double orc_echo_width_bins(const double* wf, int n, int j, double s0, double* p_out)
{
    if (p_out) p_out[0] = p_out[1] = p_out[2] = NAN;
    if (j < 0 || j >= n) return NAN;
    int L = j, R = j;
    while (L > 0 && j - L < ORC_EW_HALF && wf[L - 1] < wf[L] && 1024.0 * wf[L - 1] >= wf[j]) --L;
    while (R < n - 1 && R - j < ORC_EW_HALF && wf[R + 1] < wf[R] && 1024.0 * wf[R + 1] >= wf[j]) ++R;
    int m = R - L + 1;
    if (m < 3) return NAN;
    double x[2 * ORC_EW_HALF + 1], y[2 * ORC_EW_HALF + 1];
    for (int i = 0; i < m; ++i) {
        x[i] = (double)(L + i - j);
        y[i] = wf[L + i];
    }
    double p[3] = {wf[j], 0.0, s0};
    if (L <= j - 1 && R >= j + 1 && wf[j - 1] > 0.0 && wf[j] > 0.0 && wf[j + 1] > 0.0) {
        double lm = log(wf[j - 1]), l0 = log(wf[j]), lp = log(wf[j + 1]);
        double c2 = lm - 2.0 * l0 + lp;  /* twice the quadratic coefficient */
        if (c2 < 0.0) {
            double s2 = -1.0 / c2;
            double mu = 0.5 * (lp - lm) * s2;
            p[0] = exp(l0 + mu * mu / (2.0 * s2));
            p[1] = mu;
            p[2] = sqrt(s2);
        }
    }
    double H[6], g[3];
    double cost = ew_normal(x, y, m, p, H, g);
    double lambda = 1e-3;
    for (int it = 0; it < ORC_EW_ITERS; ++it) {
        double M[6] = {H[0] * (1.0 + lambda), H[1], H[2], H[3] * (1.0 + lambda), H[4], H[5] * (1.0 + lambda)};
        double delta[3];
        if (!ew_solve(M, g, delta)) break;
        double q[3] = {p[0] + delta[0], p[1] + delta[1], p[2] + delta[2]};
        /* a trial centre outside the lobe or a width beyond twice its length
         * counts as rejected: it heads for the flat (infinitely wide) limit */
        int inside = fabs(q[1]) <= (double)(R - L) && fabs(q[2]) <= 2.0 * (double)m;
        double cq = inside ? ew_cost(x, y, m, q) : INFINITY;
        if (cq < cost) {
            p[0] = q[0];
            p[1] = q[1];
            p[2] = q[2];
            cost = ew_normal(x, y, m, p, H, g);
            lambda *= 0.1;
        } else {
            lambda *= 10.0;
        }
    }
    if (p_out) {
        p_out[0] = p[0];
        p_out[1] = p[1];
        p_out[2] = p[2];
    }
    if (!(p[0] > 0.0) || !isfinite(p[2]) || p[2] == 0.0) return NAN;
    return fabs(p[2]);
}

/* Widths (ns) of the returns bins[0..k-1] of one waveform; the start width is
 * the pulse's own standard deviation (for Eq. 3, that of a Gaussian of the same
 * FWHM-like length). */
void orc_echo_width(const orc_scanner* sc, const double* wf, int n, const int32_t* bins, int k, double* width_ns)
{
    double s0 = gauss_sigma(sc) / sc->bin_ns;
    for (int i = 0; i < k; ++i) width_ns[i] = orc_echo_width_bins(wf, n, bins[i], s0, NULL) * sc->bin_ns;
}

/* ------------------------------------------------------------------ pulse generation (Sec. 3.2, 3.3) */

/* The paper names the platforms and deflectors and describes their patterns
 * (Sec. 3.2: a LinearPath platform moves at constant speed from one waypoint to
 * the next and always faces the next one; Sec. 3.3, Fig. 7: a polygon mirror
 * gives parallel lines of even density, a fibre array a similar pattern from
 * fixed directions, a swinging mirror a zig-zag denser at its extremes, a
 * slanted rotating (Palmer) mirror a cone at a constant angle off nadir) but no
 * formulas.  Readings taken here:
 *   time     pulse k leaves at t_k = t0 + k / prf;
 *   path     the platform covers the polyline of waypoints at `speed` from
 *            the first waypoint at t = 0 and stays at the last one afterwards;
 *            it is level and its heading (yaw) is that of the current leg's
 *            horizontal direction (one waypoint: static, heading +x);
 *   frame    platform x forward, y left, z up; world = Rz(yaw) * platform;
 *   polygon  across-track angle a = -A + 2A frac(f t) (a sawtooth);
 *   swing    a = A sin(2 pi f t);
 *   fibre    a = -A + 2A (k mod N) / (N - 1), N fibres fired in turn;
 *            for these three the direction is (0, sin a, -cos a);
 *   conic    (sin A cos p, sin A sin p, -cos A), p = 2 pi frac(f t);
 *   noise    the origin gets independent N(0, sigma^2) offsets per axis:
 *            Box-Muller on uniforms u = ((x >> 11) + 1) 2^-53 of SplitMix64
 *            output number c = 6k + 2 axis (+1) of the sequence seeded with
 *            `seed` (Steele, Lea & Flood 2014: output c mixes seed + (c + 1)
 *            times 0x9E3779B97F4A7C15).
 * The Multicopter platform (Sec. 3.2: it also speeds up and slows down; in
 * the mode without banked turns it stops at each waypoint and turns there;
 * start and end yaw of every leg may be given) is read as:
 *   legs     each leg starts from rest at its first waypoint and ends at rest
 *            at the next: constant acceleration `accel` up to `speed`, then
 *            that speed, then the same deceleration; a leg too short to reach
 *            `speed` (length below speed^2 / accel) accelerates over its first
 *            half and slows down over its second; the turn at a waypoint
 *            takes no time; afterwards the platform stays at the last one;
 *   yaw      the leg's heading, or with `leg_yaw` ([n - 1][2]: start and end
 *            yaw of each leg, rad) linear in the time spent on the leg from
 *            the start to the end value; the platform stays level.
 * The Multicopter's smooth turn mode (Sec. 3.2: the platform banks to turn
 * smoothly at the waypoints instead of stopping and turning on the spot, as
 * the banked turns of drone flight protocols do) is read as a coordinated turn:
 *   path     every interior waypoint W is cut by a circular arc tangent to
 *            both of its legs, of radius r = v^2 / (g tan b) (speed v, bank
 *            angle b, g = 9.80665 m/s^2): with u, w the unit directions into
 *            and out of W and theta = acos(u . w) the turn angle, the arc runs
 *            from W - s u to W + s w, s = r tan(theta / 2), in the plane of the
 *            two legs; the legs' straight parts join the arcs;
 *   speed    from rest at the first waypoint the platform speeds up at
 *            `accel` to v, keeps v along the straight parts and through every
 *            arc, and slows down at `accel` to rest at the last waypoint,
 *            where it stays; every leg must hold its arcs and ramps (the arc
 *            lengths s at both ends, plus v^2 / (2 accel) on the first and the
 *            last leg), and no turn may reverse a leg (theta < 179 deg);
 *   attitude heading along the horizontal direction of motion; level on the
 *            straight parts; on an arc banked by b toward the turn's centre
 *            (left when the horizontal turn is anticlockwise), the bank taken
 *            and released at the arc's ends: a platform-frame direction
 *            (x, y, z) becomes (x, y cos l + z sin l, -y sin l + z cos l) with
 *            l = +b to the left, -b to the right, then turns by the heading. */
enum { ORC_DEFLECT_POLYGON = 0, ORC_DEFLECT_SWING = 1, ORC_DEFLECT_CONIC = 2, ORC_DEFLECT_FIBRE = 3 };
enum { ORC_PLATFORM_LINEAR = 0, ORC_PLATFORM_MULTICOPTER = 1, ORC_PLATFORM_MULTICOPTER_SMOOTH = 2 };
#define ORC_G 9.80665

typedef struct {
    const double* waypoints; /* [n][3] */
    int32_t n_waypoints;
    int32_t deflector;
    double speed;            /* m/s */
    double prf;              /* pulses per second */
    double scan_freq;        /* lines (polygon), oscillations (swing), revolutions (conic) per second */
    double scan_angle;       /* A: half the line's angle, or the cone's angle off nadir (rad) */
    int32_t n_fibres;
    int32_t platform;        /* ORC_PLATFORM_* */
    double t0;
    double noise_sigma;      /* m */
    uint64_t seed;
    double accel;            /* m/s^2, Multicopter */
    const double* leg_yaw;   /* [n - 1][2] or NULL, Multicopter */
    double bank;             /* rad, Multicopter smooth turns: bank angle in (0, pi/2) */
} orc_survey;

uint64_t orc_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double sm_uniform(uint64_t seed, uint64_t c)
{
    return (double)((orc_splitmix64(seed, c) >> 11) + 1) * (1.0 / 9007199254740992.0);
}

/* Multicopter leg of length L at cruise speed v and acceleration a: its
 * duration, and the distance covered tau seconds after it starts. */
static double copter_leg_duration(double L, double v, double a)
{
    if (v * v / a <= L) return L / v + v / a; /* reaches v: two ramps of v / a, cruise over the rest */
    return 2.0 * sqrt(L / a);                  /* speeds up to sqrt(a L) half way, then slows down */
}

static double copter_leg_distance(double L, double v, double a, double T, double tau)
{
    if (tau <= 0.0) return 0.0;
    if (tau >= T) return L;
    double top = v * v / a <= L ? v : sqrt(a * L); /* highest speed on the leg */
    double ramp = top / a;                          /* time to reach it */
    if (tau <= ramp) return 0.5 * a * tau * tau;
    if (tau >= T - ramp) {
        double r = T - tau;
        return L - 0.5 * a * r * r;
    }
    return 0.5 * a * ramp * ramp + top * (tau - ramp);
}

/* The smooth turn path: its pieces in order, a straight part of each leg and an
 * arc at each interior waypoint. */
typedef struct {
    int arc;              /* 0 straight, 1 arc */
    double len;           /* arc length of the piece */
    double p0[3], dir[3]; /* straight: start point and unit direction */
    double c[3], u[3], n[3], r, lean; /* arc: centre, tangent at its start, unit vector toward the centre, radius, bank */
} orc_piece;

/* Pieces of a smooth survey; returns their number, or -1 when a leg cannot hold
 * its arcs and ramps or a turn reverses a leg.  *total gets the path length. */
static int smooth_pieces(const orc_survey* sv, orc_piece* pc, double* total)
{
    const int nw = sv->n_waypoints;
    const double v = sv->speed, r = v * v / (ORC_G * tan(sv->bank)), ramp = v * v / (2.0 * sv->accel);
    double s_at[nw > 0 ? nw : 1]; /* tangent length of the arc at each waypoint (0 at the ends) */
    double u_in[3], u_out[3];
    int np = 0;
    for (int i = 0; i < nw; ++i) s_at[i] = 0.0;
    for (int i = 1; i + 1 < nw; ++i) {
        const double *a = sv->waypoints + 3 * (i - 1), *w = sv->waypoints + 3 * i, *b = sv->waypoints + 3 * (i + 1);
        double li = 0.0, lo = 0.0, dot = 0.0;
        for (int k = 0; k < 3; ++k) {
            u_in[k] = w[k] - a[k];
            u_out[k] = b[k] - w[k];
            li += u_in[k] * u_in[k];
            lo += u_out[k] * u_out[k];
        }
        li = sqrt(li);
        lo = sqrt(lo);
        for (int k = 0; k < 3; ++k) {
            u_in[k] /= li;
            u_out[k] /= lo;
            dot += u_in[k] * u_out[k];
        }
        if (dot > 1.0) dot = 1.0;
        if (dot < -1.0) dot = -1.0;
        const double theta = acos(dot);
        if (theta > 179.0 * ORC_PI / 180.0) return -1;
        s_at[i] = r * tan(0.5 * theta);
    }
    double tot = 0.0;
    for (int j = 0; j + 1 < nw; ++j) {
        const double *a = sv->waypoints + 3 * j, *b = sv->waypoints + 3 * (j + 1);
        double d[3], L = 0.0;
        for (int k = 0; k < 3; ++k) {
            d[k] = b[k] - a[k];
            L += d[k] * d[k];
        }
        L = sqrt(L);
        for (int k = 0; k < 3; ++k) d[k] /= L;
        const double need = s_at[j] + s_at[j + 1] + (j == 0 ? ramp : 0.0) + (j + 2 == nw ? ramp : 0.0);
        if (!(need <= L)) return -1;
        /* the straight part of leg j */
        orc_piece* q = &pc[np++];
        q->arc = 0;
        q->len = L - s_at[j] - s_at[j + 1];
        for (int k = 0; k < 3; ++k) {
            q->p0[k] = a[k] + s_at[j] * d[k];
            q->dir[k] = d[k];
        }
        tot += q->len;
        if (j + 2 < nw) {
            /* the arc at waypoint j + 1 */
            const double* c2 = sv->waypoints + 3 * (j + 2);
            double w2[3], lw = 0.0, dot = 0.0;
            for (int k = 0; k < 3; ++k) {
                w2[k] = c2[k] - b[k];
                lw += w2[k] * w2[k];
            }
            lw = sqrt(lw);
            for (int k = 0; k < 3; ++k) {
                w2[k] /= lw;
                dot += d[k] * w2[k];
            }
            if (dot > 1.0) dot = 1.0;
            if (dot < -1.0) dot = -1.0;
            const double theta = acos(dot);
            if (theta > 0.0) {
                orc_piece* g = &pc[np++];
                g->arc = 1;
                g->r = r;
                g->len = r * theta;
                double nrm = 0.0;
                for (int k = 0; k < 3; ++k) {
                    g->n[k] = w2[k] - dot * d[k];
                    nrm += g->n[k] * g->n[k];
                }
                nrm = sqrt(nrm);
                for (int k = 0; k < 3; ++k) {
                    g->n[k] /= nrm;
                    g->u[k] = d[k];
                    g->c[k] = b[k] - s_at[j + 1] * d[k] + r * g->n[k];
                }
                /* bank toward the centre: left for an anticlockwise horizontal turn */
                const double turn_z = d[0] * w2[1] - d[1] * w2[0];
                g->lean = turn_z > 0.0 ? sv->bank : (turn_z < 0.0 ? -sv->bank : 0.0);
                tot += g->len;
            }
        }
    }
    *total = tot;
    return np;
}

/* Position, unit direction of motion and bank of the smooth path at path length
 * sigma (0 <= sigma <= total). */
static void smooth_at(const orc_piece* pc, int np, double sigma, double* pos, double* dir, double* lean)
{
    int i = 0;
    while (i + 1 < np && sigma > pc[i].len) {
        sigma -= pc[i].len;
        ++i;
    }
    const orc_piece* q = &pc[i];
    if (sigma > q->len) sigma = q->len;
    if (!q->arc) {
        for (int k = 0; k < 3; ++k) {
            pos[k] = q->p0[k] + sigma * q->dir[k];
            dir[k] = q->dir[k];
        }
        *lean = 0.0;
        return;
    }
    const double ph = sigma / q->r;
    for (int k = 0; k < 3; ++k) {
        pos[k] = q->c[k] - q->r * cos(ph) * q->n[k] + q->r * sin(ph) * q->u[k];
        dir[k] = cos(ph) * q->u[k] + sin(ph) * q->n[k];
    }
    *lean = q->lean;
}

/* Pulses [first, first + count): origins [count][3], directions [count][3]
 * (unit, FP64).  Returns 0, or -1 for an invalid survey. */
int orc_generate_pulses(const orc_survey* sv, int64_t first, int64_t count, double* origins, double* dirs)
{
    int nw = sv->n_waypoints;
    if (nw < 1 || !(sv->prf > 0.0)) return -1;
    if (sv->deflector == ORC_DEFLECT_FIBRE && sv->n_fibres < 2) return -1;
    int copter = sv->platform == ORC_PLATFORM_MULTICOPTER;
    int smooth = sv->platform == ORC_PLATFORM_MULTICOPTER_SMOOTH;
    if (sv->platform != ORC_PLATFORM_LINEAR && !copter && !smooth) return -1;
    if ((copter || smooth) && nw >= 2 && !(sv->speed > 0.0 && sv->accel > 0.0)) return -1;
    if (!copter && sv->leg_yaw) return -1;
    if (smooth && !(sv->bank > 0.0 && sv->bank < 0.5 * ORC_PI)) return -1;
    orc_piece* pc = NULL;
    int np = 0;
    double total = 0.0, T_end = 0.0;
    if (smooth && nw >= 2) {
        pc = (orc_piece*)malloc(sizeof(orc_piece) * (size_t)(2 * nw));
        for (int i = 1; i < nw; ++i) {
            const double *a = sv->waypoints + 3 * (i - 1), *b = sv->waypoints + 3 * i;
            if (!((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]) > 0.0)) {
                free(pc);
                return -1;
            }
        }
        np = smooth_pieces(sv, pc, &total);
        if (np < 0) {
            free(pc);
            return -1;
        }
        T_end = total / sv->speed + sv->speed / sv->accel;
    }
    double* cum = (double*)malloc(sizeof(double) * (size_t)nw);   /* path length at each waypoint */
    double* start = (double*)malloc(sizeof(double) * (size_t)nw); /* Multicopter: time at each waypoint */
    cum[0] = 0.0;
    start[0] = 0.0;
    for (int i = 1; i < nw; ++i) {
        const double* a = sv->waypoints + 3 * (i - 1);
        const double* b = sv->waypoints + 3 * i;
        double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
        double len = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(len > 0.0)) { /* consecutive waypoints must differ */
            free(cum);
            free(start);
            return -1;
        }
        cum[i] = cum[i - 1] + len;
        start[i] = copter ? start[i - 1] + copter_leg_duration(len, sv->speed, sv->accel) : 0.0;
    }
    for (int64_t q = 0; q < count; ++q) {
        int64_t k = first + q;
        double t = sv->t0 + (double)k / sv->prf;
        /* position along the path and heading of the current leg */
        double pos[3] = {sv->waypoints[0], sv->waypoints[1], sv->waypoints[2]};
        double yaw = 0.0, lean = 0.0;
        if (nw >= 2 && smooth) {
            /* path length covered: ramp up, cruise, ramp down (Sec. 3.2 reading above) */
            const double v = sv->speed, acc = sv->accel, tr = v / acc;
            double sigma;
            if (t <= 0.0) sigma = 0.0;
            else if (t <= tr) sigma = 0.5 * acc * t * t;
            else if (t < T_end - tr) sigma = 0.5 * acc * tr * tr + v * (t - tr);
            else if (t < T_end) sigma = total - 0.5 * acc * (T_end - t) * (T_end - t);
            else sigma = total;
            double dir[3];
            smooth_at(pc, np, sigma, pos, dir, &lean);
            yaw = atan2(dir[1], dir[0]);
        } else if (nw >= 2 && copter) {
            int leg = 0;
            while (leg + 2 < nw && start[leg + 1] <= t) ++leg;
            const double* a = sv->waypoints + 3 * leg;
            const double* b = sv->waypoints + 3 * (leg + 1);
            double L = cum[leg + 1] - cum[leg];
            double T = start[leg + 1] - start[leg];
            double tau = t - start[leg];
            if (tau < 0.0) tau = 0.0;
            if (tau > T) tau = T;
            double f = copter_leg_distance(L, sv->speed, sv->accel, T, tau) / L;
            for (int i = 0; i < 3; ++i) pos[i] = a[i] + f * (b[i] - a[i]);
            if (sv->leg_yaw) {
                double y0 = sv->leg_yaw[2 * leg], y1 = sv->leg_yaw[2 * leg + 1];
                yaw = y0 + (tau / T) * (y1 - y0);
            } else {
                yaw = atan2(b[1] - a[1], b[0] - a[0]);
            }
        } else if (nw >= 2) {
            double sdist = sv->speed * t;
            int leg = 0;
            while (leg + 2 < nw && cum[leg + 1] <= sdist) ++leg;
            const double* a = sv->waypoints + 3 * leg;
            const double* b = sv->waypoints + 3 * (leg + 1);
            double len = cum[leg + 1] - cum[leg];
            double f = len > 0.0 ? (sdist - cum[leg]) / len : 0.0;
            if (f < 0.0) f = 0.0;
            if (f > 1.0) f = 1.0;
            for (int i = 0; i < 3; ++i) pos[i] = a[i] + f * (b[i] - a[i]);
            yaw = atan2(b[1] - a[1], b[0] - a[0]);
        }
        if (sv->noise_sigma > 0.0) {
            for (int ax = 0; ax < 3; ++ax) {
                uint64_t c = 6 * (uint64_t)k + 2 * (uint64_t)ax;
                double u1 = sm_uniform(sv->seed, c), u2 = sm_uniform(sv->seed, c + 1);
                pos[ax] += sv->noise_sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
            }
        }
        /* direction in the platform frame */
        double A = sv->scan_angle, d[3];
        double ph = sv->scan_freq * t;
        ph -= floor(ph);
        if (sv->deflector == ORC_DEFLECT_CONIC) {
            double p = 2.0 * ORC_PI * ph;
            d[0] = sin(A) * cos(p);
            d[1] = sin(A) * sin(p);
            d[2] = -cos(A);
        } else {
            double ang;
            if (sv->deflector == ORC_DEFLECT_POLYGON) ang = -A + 2.0 * A * ph;
            else if (sv->deflector == ORC_DEFLECT_SWING) ang = A * sin(2.0 * ORC_PI * sv->scan_freq * t);
            else ang = -A + 2.0 * A * (double)(k % sv->n_fibres) / (double)(sv->n_fibres - 1);
            d[0] = 0.0;
            d[1] = sin(ang);
            d[2] = -cos(ang);
        }
        if (lean != 0.0) {
            /* banked toward the turn's centre */
            double cl = cos(lean), sl = sin(lean);
            double y = d[1] * cl + d[2] * sl, z = -d[1] * sl + d[2] * cl;
            d[1] = y;
            d[2] = z;
        }
        double cy = cos(yaw), sy = sin(yaw);
        double* o = origins + 3 * q;
        double* w = dirs + 3 * q;
        for (int i = 0; i < 3; ++i) o[i] = pos[i];
        w[0] = cy * d[0] - sy * d[1];
        w[1] = sy * d[0] + cy * d[1];
        w[2] = d[2];
    }
    free(cum);
    free(start);
    free(pc);
    return 0;
}

/* Scene parts (Sec. 3.5, Sec. 5.1): instance vertices x -> A x + t with A and t
 * the rows [A_i0 A_i1 A_i2 t_i] of `affine` (row-major 3 x 4), evaluated in
 * FP64 in that order and rounded once to FP32. */
void orc_instance_vertices(const float* v, int64_t nv, const double affine[12], float* out)
{
    for (int64_t q = 0; q < nv; ++q) {
        double x = v[3 * q], y = v[3 * q + 1], z = v[3 * q + 2];
        for (int i = 0; i < 3; ++i) {
            const double* r = affine + 4 * i;
            double w = r[0] * x;
            w = w + r[1] * y;
            w = w + r[2] * z;
            w = w + r[3];
            out[3 * q + i] = (float)w;
        }
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
