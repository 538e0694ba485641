/*
 * oracle.c -- plain, slow CPU reference of the seed-scan hot path, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY. It is used by the test suite, by the smoke check and
 * by the benchmark's CPU-baseline leg, and by nothing else. It shares no code,
 * header, table or helper with the GPU library; the two meet only through the
 * written evaluation-order contract below and the seeded synthetic inputs.
 *
 * What it computes (paper: "GPU-accelerated event reconstruction for the COMET
 * Phase-I experiment", arXiv:1911.09340):
 *   - seeds on a grid over prior ranges of the seed components     (Sec. 2.1, Sec. 3.1)
 *   - a track recorded from every seed by Runge-Kutta stepping     (Sec. 2.2.1, Alg. 1)
 *   - per wire, the recorded state closest to the wire, refined
 *     locally to the distance of closest approach (DCA)             (Sec. 2.2.2, Alg. 2)
 *   - the residual sum of squares of the lambda-capped DCA residual (Sec. 2.1, Eq. 1)
 *   - one thread per seed doing both steps, as the CPU scheme does  (Sec. 2.3, Alg. 3)
 *   - the lowest-RSS seed, a finer re-scan around it, and the hits
 *     whose residual is below lambda                                (Sec. 2.1)
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - uniform field B = (0, 0, bz), fixed-step classical RK4 in path length with
 *     |p| held constant (the paper uses adaptive RKN in a field map);
 *   - the left/right hits of a drift circle of radius r around a wire whose DCA
 *     to the track is D have DCAs |D - r| and D + r, so min(dL, dR) = |D - r|;
 *   - the local refinement from the closest recorded point is the exact minimum
 *     over the two chords adjacent to it (the paper iterates RKN steps towards a
 *     plane through the wire until a tolerance);
 *   - wires are infinite lines through their two endpoints.
 *
 * Evaluation-order contract. Every formula is evaluated exactly as written here
 * (the file is built with -ffp-contract=off); fma() appears only where written.
 * Division and square root are the correctly rounded IEEE operations.
 *
 * Units: mm, MeV/c, tesla, charge in units of e.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_KAPPA 0.299792458 /* MeV/c per (T mm) */

/* ------------------------------------------------------------ seed grid
 * Sec. 3.1: a seed set is the product of grids over the prior range of each
 * seed component. Here the four axes are (arc offset along the seed circle,
 * |p|, polar-angle offset, azimuth offset) around a reference state; axis 3 runs
 * fastest. grid = ref[6], centre[4], half[4].
 *
 * Axis value i of n: centre (n == 1) or centre + half * ((2i - (n-1)) / (n-1)).
 * An offset v turns into a rotation through the half-angle tangent tau:
 * cos = (1 - tau^2) / (1 + tau^2), sin = (2 tau) / (1 + tau^2); tau = v / (2 r0)
 * for the arc offset (r0 = the reference radius), tau = v / 2 for the angles, so
 * the rotation angle is 2 atan(tau) (within 4e-4 of v for the spans used).
 */
double oracle_axis_value(double centre, double half, int32_t n, int32_t i)
{
    if (n == 1)
        return centre;
    return centre + half * ((double)(2 * i - (n - 1)) / (double)(n - 1));
}

static void half_angle_rotation(double tau, double *c, double *s)
{
    double t2 = tau * tau;
    double den = 1.0 + t2;
    *c = (1.0 - t2) / den;
    *s = (2.0 * tau) / den;
}

void oracle_seed(const double grid[14], const int32_t n[4], int64_t index, double out[6])
{
    const double *ref = grid, *ctr = grid + 6, *half = grid + 10;
    int32_t i3 = (int32_t)(index % n[3]);
    int64_t rest = index / n[3];
    int32_t i2 = (int32_t)(rest % n[2]);
    rest /= n[2];
    int32_t i1 = (int32_t)(rest % n[1]);
    int32_t i0 = (int32_t)(rest / n[1]);
    double v0 = oracle_axis_value(ctr[0], half[0], n[0], i0);
    double v1 = oracle_axis_value(ctr[1], half[1], n[1], i1);
    double v2 = oracle_axis_value(ctr[2], half[2], n[2], i2);
    double v3 = oracle_axis_value(ctr[3], half[3], n[3], i3);

    double x0 = ref[0], y0 = ref[1], z0 = ref[2];
    double px0 = ref[3], py0 = ref[4], pz0 = ref[5];
    double r0 = sqrt(x0 * x0 + y0 * y0);
    double ca, sa;
    half_angle_rotation(v0 / (2.0 * r0), &ca, &sa);
    out[0] = x0 * ca - y0 * sa;
    out[1] = y0 * ca + x0 * sa;
    out[2] = z0;

    double pt0 = sqrt(px0 * px0 + py0 * py0);
    double p0 = sqrt((px0 * px0 + py0 * py0) + pz0 * pz0);
    double ct0 = pz0 / p0, st0 = pt0 / p0;
    double cp0 = px0 / pt0, sp0 = py0 / pt0;
    double cdt, sdt, cdp, sdp;
    half_angle_rotation(v2 * 0.5, &cdt, &sdt);
    half_angle_rotation(v3 * 0.5, &cdp, &sdp);
    double ct = ct0 * cdt - st0 * sdt;
    double st = st0 * cdt + ct0 * sdt;
    double cp = cp0 * cdp - sp0 * sdp;
    double sp = sp0 * cdp + cp0 * sdp;
    out[3] = v1 * (st * cp);
    out[4] = v1 * (st * sp);
    out[5] = v1 * ct;
}

/* seeds: SoA [6][S], S = n0 n1 n2 n3 */
void oracle_seed_grid(const double grid[14], const int32_t n[4], double *seeds)
{
    int64_t S = (int64_t)n[0] * n[1] * n[2] * n[3];
    for (int64_t s = 0; s < S; ++s) {
        double st[6];
        oracle_seed(grid, n, s, st);
        for (int c = 0; c < 6; ++c)
            seeds[c * S + s] = st[c];
    }
}

/* Sec. 2.1 (finer re-scan around the best seed): each axis with n > 1 is
 * re-centred on the best seed's value and its half-span becomes one spacing of
 * the previous grid, 2 half / (n - 1). */
void oracle_refine_grid(double grid[14], const int32_t n[4], int64_t best)
{
    if (best < 0)
        return;
    int32_t idx[4];
    int64_t rest = best;
    for (int a = 3; a >= 0; --a) {
        idx[a] = (int32_t)(rest % n[a]);
        rest /= n[a];
    }
    for (int a = 0; a < 4; ++a) {
        if (n[a] > 1) {
            double v = oracle_axis_value(grid[6 + a], grid[10 + a], n[a], idx[a]);
            grid[6 + a] = v;
            grid[10 + a] = (2.0 * grid[10 + a]) / (double)(n[a] - 1);
        }
    }
}

/* ------------------------------------------------------------ track recording
 * Alg. 1 / Sec. 2.2.1: the state is stepped and every position is recorded.
 * ODE in path length s for y = (x, p): dx/ds = p / p0, dp/ds = c (p_y, -p_x, 0)
 * with p0 = |p| of the seed and c = KAPPA q bz / p0 (uniform field along z;
 * p_z never changes). Classical RK4 with fixed step h, K steps, K+1 points:
 *   k1 = f(y), k2 = f(y + h/2 k1), k3 = f(y + h/2 k2), k4 = f(y + h k3),
 *   y <- y + h/6 (((k1 + 2 k2) + 2 k3) + k4).
 * pts: AoS [K+1][3].
 */
typedef struct {
    double inv, c, h, hh, h6, vz;
} rk4_consts;

static rk4_consts rk4_setup(double px, double py, double pz, double bz, double charge, double h)
{
    rk4_consts k;
    double p0 = sqrt((px * px + py * py) + pz * pz);
    k.inv = 1.0 / p0;
    k.c = ((ORACLE_KAPPA * charge) * bz) * k.inv;
    k.h = h;
    k.hh = 0.5 * h;
    k.h6 = h / 6.0;
    k.vz = pz * k.inv; /* z velocity: the same at every stage */
    return k;
}

/* one RK4 step of (x, y, z, px, py); p_z is constant */
static void rk4_step(const rk4_consts *k, double *x, double *y, double *z, double *px,
                     double *py)
{
    const double inv = k->inv, c = k->c, h = k->h, hh = k->hh, h6 = k->h6, vz = k->vz;
    /* stage 1 at p */
    double v1x = *px * inv, v1y = *py * inv;
    double f1x = c * *py, f1y = -(c * *px);
    /* stage 2 at p + h/2 f1 */
    double qx = *px + hh * f1x, qy = *py + hh * f1y;
    double v2x = qx * inv, v2y = qy * inv;
    double f2x = c * qy, f2y = -(c * qx);
    /* stage 3 at p + h/2 f2 */
    qx = *px + hh * f2x;
    qy = *py + hh * f2y;
    double v3x = qx * inv, v3y = qy * inv;
    double f3x = c * qy, f3y = -(c * qx);
    /* stage 4 at p + h f3 */
    qx = *px + h * f3x;
    qy = *py + h * f3y;
    double v4x = qx * inv, v4y = qy * inv;
    double f4x = c * qy, f4y = -(c * qx);

    *x = *x + h6 * (((v1x + 2.0 * v2x) + 2.0 * v3x) + v4x);
    *y = *y + h6 * (((v1y + 2.0 * v2y) + 2.0 * v3y) + v4y);
    *z = *z + h6 * (((vz + 2.0 * vz) + 2.0 * vz) + vz);
    *px = *px + h6 * (((f1x + 2.0 * f2x) + 2.0 * f3x) + f4x);
    *py = *py + h6 * (((f1y + 2.0 * f2y) + 2.0 * f3y) + f4y);
}

void oracle_track(const double seed[6], double bz, double charge, double h, int32_t K,
                  double *pts)
{
    double x = seed[0], y = seed[1], z = seed[2];
    double px = seed[3], py = seed[4];
    const rk4_consts k = rk4_setup(px, py, seed[5], bz, charge, h);
    for (int32_t j = 0; j < K; ++j) {
        pts[3 * j + 0] = x;
        pts[3 * j + 1] = y;
        pts[3 * j + 2] = z;
        rk4_step(&k, &x, &y, &z, &px, &py);
    }
    pts[3 * K + 0] = x;
    pts[3 * K + 1] = y;
    pts[3 * K + 2] = z;
}

/* ------------------------------------------------------------ wire frame
 * Alg. 2 keeps both endpoints of a wire. The distance of a point P to the wire
 * line is the length of P - A projected on the plane normal to the unit wire
 * direction n. That plane is spanned by an orthonormal pair (e1, e2) built from n
 * with the branch-free construction of Duff et al., "Building an orthonormal
 * basis, revisited" (JCGT 2017):
 *   s = copysign(1, n_z), a = -1 / (s + n_z), b = (n_x n_y) a,
 *   e1 = (1 + ((s n_x) n_x) a, s b, -(s n_x)),  e2 = (b, s + (n_y n_y) a, -n_y).
 * frame = (e1x, e1y, e1z, -c1, e2x, e2y, e2z, -c2) with c = (e_x A_x + e_y A_y) + e_z A_z.
 */
void oracle_wire_frame(const double ends[6], double frame[8])
{
    double ax = ends[0], ay = ends[1], az = ends[2];
    double dx = ends[3] - ax, dy = ends[4] - ay, dz = ends[5] - az;
    double len = sqrt((dx * dx + dy * dy) + dz * dz);
    double nx = dx / len, ny = dy / len, nz = dz / len;
    double s = copysign(1.0, nz);
    double a = -1.0 / (s + nz);
    double b = (nx * ny) * a;
    double e1x = 1.0 + ((s * nx) * nx) * a, e1y = s * b, e1z = -(s * nx);
    double e2x = b, e2y = s + (ny * ny) * a, e2z = -ny;
    frame[0] = e1x;
    frame[1] = e1y;
    frame[2] = e1z;
    frame[3] = -((e1x * ax + e1y * ay) + e1z * az);
    frame[4] = e2x;
    frame[5] = e2y;
    frame[6] = e2z;
    frame[7] = -((e2x * ax + e2y * ay) + e2z * az);
}

/* In-plane coordinates of P relative to the wire:
 * xi = fma(e1x, x, fma(e1y, y, fma(e1z, z, -c1))), eta likewise with e2. */
static void project(const double f[8], const double *p, double *xi, double *eta)
{
    *xi = fma(f[0], p[0], fma(f[1], p[1], fma(f[2], p[2], f[3])));
    *eta = fma(f[4], p[0], fma(f[5], p[1], fma(f[6], p[2], f[7])));
}

/* Squared distance from the wire to the chord a -> b (in-plane coordinates):
 * u = b - a, g = fma(a_xi, u_xi, a_eta u_eta), den = fma(u_xi, u_xi, u_eta u_eta);
 * t = clamp(-g / den, 0, 1): t = 0 (g >= 0) gives qa, t = 1 (-g >= den) gives qb,
 * otherwise the point a + t u gives fma(p_xi, p_xi, p_eta p_eta). */
static double chord_distance2(double axi, double aeta, double qa, double bxi, double beta,
                              double qb)
{
    double uxi = bxi - axi, ueta = beta - aeta;
    double g = fma(axi, uxi, aeta * ueta);
    double den = fma(uxi, uxi, ueta * ueta);
    if (!(g < 0.0))
        return qa;
    if (-g >= den)
        return qb;
    double t = -g / den;
    double pxi = fma(t, uxi, axi), peta = fma(t, ueta, aeta);
    return fma(pxi, pxi, peta * peta);
}

/* Alg. 2 / Alg. 3: find the recorded point closest to the wire (first index of
 * the minimum of q_k = fma(xi, xi, eta eta)), then refine over its two adjacent
 * chords. Returns the squared DCA; *kstar receives the closest point's index.
 * pts: AoS [P][3], P >= 2. */
double oracle_dca2(const double *pts, int32_t P, const double frame[8], int32_t *kstar)
{
    int32_t kb = 0;
    double qb = INFINITY;
    for (int32_t k = 0; k < P; ++k) {
        double xi, eta;
        project(frame, pts + 3 * k, &xi, &eta);
        double q = fma(xi, xi, eta * eta);
        if (q < qb) {
            qb = q;
            kb = k;
        }
    }
    double cxi, ceta;
    project(frame, pts + 3 * kb, &cxi, &ceta);
    double d2 = qb;
    if (kb > 0) {
        double xi, eta;
        project(frame, pts + 3 * (kb - 1), &xi, &eta);
        double q = fma(xi, xi, eta * eta);
        double v = chord_distance2(xi, eta, q, cxi, ceta, qb);
        if (v < d2)
            d2 = v;
    }
    if (kb < P - 1) {
        double xi, eta;
        project(frame, pts + 3 * (kb + 1), &xi, &eta);
        double q = fma(xi, xi, eta * eta);
        double v = chord_distance2(cxi, ceta, qb, xi, eta, q);
        if (v < d2)
            d2 = v;
    }
    if (kstar)
        *kstar = kb;
    return d2;
}

/* Eq. 1: d_i = min(min_j |D_i - r_j|, lambda) over the hits j of wire i (a wire
 * without hits gives lambda), RSS = sum over wires in order of d_i^2. */
static double wire_residual(double D, const double *drift, int32_t j0, int32_t j1,
                            double lambda)
{
    double d = lambda;
    for (int32_t j = j0; j < j1; ++j) {
        double e = fabs(D - drift[j]);
        if (e < d)
            d = e;
    }
    return d;
}

double oracle_rss_track(const double *pts, int32_t P, const double *frames, int32_t n_wires,
                        const int32_t *offsets, const double *drift, double lambda)
{
    double rss = 0.0;
    for (int32_t i = 0; i < n_wires; ++i) {
        double D = sqrt(oracle_dca2(pts, P, frames + 8 * i, NULL));
        double d = wire_residual(D, drift, offsets[i], offsets[i + 1], lambda);
        rss = rss + d * d;
    }
    return rss;
}

/* Alg. 3: one thread per seed records its track and sums Eq. 1 over the wires.
 * seeds: SoA [6][S]. cfg = (bz, charge, h, lambda). Returns the threads used. */
int32_t oracle_scan(const double *seeds, int64_t S, const double cfg[4], int32_t K,
                    const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                    const double *drift, double *rss, int32_t n_threads)
{
    double *frames = (double *)malloc(sizeof(double) * 8 * (size_t)(n_wires > 0 ? n_wires : 1));
    for (int32_t i = 0; i < n_wires; ++i)
        oracle_wire_frame(wire_ends + 6 * i, frames + 8 * i);
    int32_t used = 1;
#ifdef _OPENMP
    if (n_threads <= 0)
        n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
    {
#pragma omp single
        used = omp_get_num_threads();
        double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t s = 0; s < S; ++s) {
            double seed[6];
            for (int c = 0; c < 6; ++c)
                seed[c] = seeds[c * S + s];
            oracle_track(seed, cfg[0], cfg[1], cfg[2], K, pts);
            rss[s] = oracle_rss_track(pts, K + 1, frames, n_wires, offsets, drift, cfg[3]);
        }
        free(pts);
    }
#else
    (void)n_threads;
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
    for (int64_t s = 0; s < S; ++s) {
        double seed[6];
        for (int c = 0; c < 6; ++c)
            seed[c] = seeds[c * S + s];
        oracle_track(seed, cfg[0], cfg[1], cfg[2], K, pts);
        rss[s] = oracle_rss_track(pts, K + 1, frames, n_wires, offsets, drift, cfg[3]);
    }
    free(pts);
#endif
    free(frames);
    return used;
}

/* Lowest RSS; ties go to the lowest index; NaN is never chosen (-1 if all are). */
int64_t oracle_argmin(const double *rss, int64_t S)
{
    int64_t b = -1;
    double v = INFINITY;
    for (int64_t s = 0; s < S; ++s) {
        if (rss[s] < v || (b < 0 && rss[s] == v)) {
            v = rss[s];
            b = s;
        }
    }
    return b;
}

/* Sec. 2.1, classification: on every wire the hit with the smallest |D - r_j|
 * (lowest index on ties) is the track's when that residual is below lambda
 * (strictly). mask[j]: bit 0 = classified, bit 1 = borderline (the wire's closest
 * hit has ||D - r| - lambda| < 1e-9 mm). dca[i] receives D_i (may be NULL).
 * Returns the number of borderline hits. */
static int32_t classify_track(const double *pts, int32_t K, const double cfg[4],
                              const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                              const double *drift, uint8_t *mask, double *dca)
{
    int32_t n_border = 0;
    for (int32_t i = 0; i < n_wires; ++i) {
        double frame[8];
        oracle_wire_frame(wire_ends + 6 * i, frame);
        double D = sqrt(oracle_dca2(pts, K + 1, frame, NULL));
        if (dca)
            dca[i] = D;
        int32_t jb = -1;
        double eb = INFINITY;
        for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j) {
            mask[j] = 0;
            double e = fabs(D - drift[j]);
            if (e < eb) {
                eb = e;
                jb = j;
            }
        }
        if (jb >= 0) {
            uint8_t m = 0;
            if (eb < cfg[3])
                m |= 1;
            if (fabs(eb - cfg[3]) < 1e-9) {
                m |= 2;
                n_border += 1;
            }
            mask[jb] = m;
        }
    }
    return n_border;
}

int32_t oracle_classify(const double seed[6], const double cfg[4], int32_t K,
                        const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                        const double *drift, uint8_t *mask, double *dca)
{
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
    oracle_track(seed, cfg[0], cfg[1], cfg[2], K, pts);
    int32_t n_border = classify_track(pts, K, cfg, wire_ends, n_wires, offsets, drift, mask,
                                      dca);
    free(pts);
    return n_border;
}

/* The whole path for one turn partition: scan the grid, then n_refine finer
 * re-scans around the best seed (Sec. 2.1), then classify at the final best.
 * grid is updated in place; rss_out receives the last scan's RSS [S] (may be NULL).
 * best_seed[6], best_rss[1] and the hit mask are outputs. Returns the best index
 * in the last grid. */
int64_t oracle_scan_partition(double grid[14], const int32_t n[4], const double cfg[4],
                              int32_t K, int32_t n_refine, const double *wire_ends,
                              int32_t n_wires, const int32_t *offsets, const double *drift,
                              double *rss_out, double *best_seed, double *best_rss,
                              uint8_t *mask, int32_t *n_border, int32_t n_threads)
{
    int64_t S = (int64_t)n[0] * n[1] * n[2] * n[3];
    double *seeds = (double *)malloc(sizeof(double) * 6 * (size_t)S);
    double *rss = rss_out ? rss_out : (double *)malloc(sizeof(double) * (size_t)S);
    int64_t b = -1;
    for (int32_t it = 0; it <= n_refine; ++it) {
        if (it > 0)
            oracle_refine_grid(grid, n, b);
        oracle_seed_grid(grid, n, seeds);
        oracle_scan(seeds, S, cfg, K, wire_ends, n_wires, offsets, drift, rss, n_threads);
        b = oracle_argmin(rss, S);
    }
    if (b >= 0) {
        oracle_seed(grid, n, b, best_seed);
        *best_rss = rss[b];
        int32_t nb = oracle_classify(best_seed, cfg, K, wire_ends, n_wires, offsets, drift,
                                     mask, NULL);
        if (n_border)
            *n_border = nb;
    }
    free(seeds);
    if (!rss_out)
        free(rss);
    return b;
}

/* ------------------------------------------------------------ derivatives
 * Forward-mode dual numbers: every quantity carries its value and its derivatives
 * with respect to the six seed components (x, y, z, px, py, pz). The value parts are
 * computed with exactly the operations above, so closest points, chords and hits
 * are chosen as in the plain functions; the derivative parts follow the chain rule
 * of each operation. This is the oracle of the GPU adjoint (reverse mode), which
 * shares nothing with it but the mathematics. */
typedef struct {
    double v;
    double d[6];
} dual;

static dual dc(double v)
{
    dual r;
    r.v = v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = 0.0;
    return r;
}

static dual dvar(double v, int i)
{
    dual r = dc(v);
    r.d[i] = 1.0;
    return r;
}

static dual dadd(dual a, dual b)
{
    dual r;
    r.v = a.v + b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] + b.d[i];
    return r;
}

static dual dsub(dual a, dual b)
{
    dual r;
    r.v = a.v - b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] - b.d[i];
    return r;
}

static dual dneg(dual a)
{
    dual r;
    r.v = -a.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = -a.d[i];
    return r;
}

static dual dmul(dual a, dual b)
{
    dual r;
    r.v = a.v * b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}

static dual ddiv(dual a, dual b)
{
    dual r;
    r.v = a.v / b.v;
    for (int i = 0; i < 6; ++i)
        r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}

static dual dsqrt(dual a)
{
    dual r;
    r.v = sqrt(a.v);
    for (int i = 0; i < 6; ++i)
        r.d[i] = r.v > 0.0 ? a.d[i] / (2.0 * r.v) : 0.0;
    return r;
}

/* fma(a, b, c): value rounded once, derivative a' b + a b' + c' */
static dual dfma(dual a, dual b, dual c)
{
    dual r;
    r.v = fma(a.v, b.v, c.v);
    for (int i = 0; i < 6; ++i)
        r.d[i] = a.d[i] * b.v + a.v * b.d[i] + c.d[i];
    return r;
}

/* RK4 track of the seed in dual numbers; pts: [K+1][3] duals. */
static void dual_track(const double seed[6], double bz, double charge, double h, int32_t K,
                       dual *pts)
{
    dual x = dvar(seed[0], 0), y = dvar(seed[1], 1), z = dvar(seed[2], 2);
    dual px = dvar(seed[3], 3), py = dvar(seed[4], 4), pz = dvar(seed[5], 5);
    dual p0 = dsqrt(dadd(dadd(dmul(px, px), dmul(py, py)), dmul(pz, pz)));
    dual inv = ddiv(dc(1.0), p0);
    dual c = dmul(dc((ORACLE_KAPPA * charge) * bz), inv);
    dual hh = dc(0.5 * h), hd = dc(h), h6 = dc(h / 6.0), two = dc(2.0);
    dual vz = dmul(pz, inv);
    for (int32_t k = 0; k < K; ++k) {
        pts[3 * k + 0] = x;
        pts[3 * k + 1] = y;
        pts[3 * k + 2] = z;
        dual v1x = dmul(px, inv), v1y = dmul(py, inv);
        dual f1x = dmul(c, py), f1y = dneg(dmul(c, px));
        dual qx = dadd(px, dmul(hh, f1x)), qy = dadd(py, dmul(hh, f1y));
        dual v2x = dmul(qx, inv), v2y = dmul(qy, inv);
        dual f2x = dmul(c, qy), f2y = dneg(dmul(c, qx));
        qx = dadd(px, dmul(hh, f2x));
        qy = dadd(py, dmul(hh, f2y));
        dual v3x = dmul(qx, inv), v3y = dmul(qy, inv);
        dual f3x = dmul(c, qy), f3y = dneg(dmul(c, qx));
        qx = dadd(px, dmul(hd, f3x));
        qy = dadd(py, dmul(hd, f3y));
        dual v4x = dmul(qx, inv), v4y = dmul(qy, inv);
        dual f4x = dmul(c, qy), f4y = dneg(dmul(c, qx));
        x = dadd(x, dmul(h6, dadd(dadd(dadd(v1x, dmul(two, v2x)), dmul(two, v3x)), v4x)));
        y = dadd(y, dmul(h6, dadd(dadd(dadd(v1y, dmul(two, v2y)), dmul(two, v3y)), v4y)));
        z = dadd(z, dmul(h6, dadd(dadd(dadd(vz, dmul(two, vz)), dmul(two, vz)), vz)));
        px = dadd(px, dmul(h6, dadd(dadd(dadd(f1x, dmul(two, f2x)), dmul(two, f3x)), f4x)));
        py = dadd(py, dmul(h6, dadd(dadd(dadd(f1y, dmul(two, f2y)), dmul(two, f3y)), f4y)));
    }
    pts[3 * K + 0] = x;
    pts[3 * K + 1] = y;
    pts[3 * K + 2] = z;
}

static void dual_project(const double f[8], const dual *p, dual *xi, dual *eta)
{
    *xi = dfma(dc(f[0]), p[0], dfma(dc(f[1]), p[1], dfma(dc(f[2]), p[2], dc(f[3]))));
    *eta = dfma(dc(f[4]), p[0], dfma(dc(f[5]), p[1], dfma(dc(f[6]), p[2], dc(f[7]))));
}

static dual dual_chord(dual axi, dual aeta, dual qa, dual bxi, dual beta, dual qb)
{
    dual uxi = dsub(bxi, axi), ueta = dsub(beta, aeta);
    dual g = dfma(axi, uxi, dmul(aeta, ueta));
    dual den = dfma(uxi, uxi, dmul(ueta, ueta));
    if (!(g.v < 0.0))
        return qa;
    if (-g.v >= den.v)
        return qb;
    dual t = ddiv(dneg(g), den);
    dual pxi = dfma(t, uxi, axi), peta = dfma(t, ueta, aeta);
    return dfma(pxi, pxi, dmul(peta, peta));
}

/* The squared DCA of one wire in dual numbers (same choices as oracle_dca2). */
static dual dual_dca2(const dual *pts, int32_t P, const double frame[8])
{
    int32_t kb = 0;
    double qbv = INFINITY;
    for (int32_t k = 0; k < P; ++k) {
        double xi, eta;
        double pv[3] = {pts[3 * k].v, pts[3 * k + 1].v, pts[3 * k + 2].v};
        project(frame, pv, &xi, &eta);
        double q = fma(xi, xi, eta * eta);
        if (q < qbv) {
            qbv = q;
            kb = k;
        }
    }
    dual cxi, ceta;
    dual_project(frame, pts + 3 * kb, &cxi, &ceta);
    dual qb = dfma(cxi, cxi, dmul(ceta, ceta));
    dual d2 = qb;
    if (kb > 0) {
        dual xi, eta;
        dual_project(frame, pts + 3 * (kb - 1), &xi, &eta);
        dual q = dfma(xi, xi, dmul(eta, eta));
        dual v = dual_chord(xi, eta, q, cxi, ceta, qb);
        if (v.v < d2.v)
            d2 = v;
    }
    if (kb < P - 1) {
        dual xi, eta;
        dual_project(frame, pts + 3 * (kb + 1), &xi, &eta);
        dual q = dfma(xi, xi, dmul(eta, eta));
        dual v = dual_chord(cxi, ceta, qb, xi, eta, q);
        if (v.v < d2.v)
            d2 = v;
    }
    return d2;
}

/* Per wire: D_i and its derivatives J_i = dD_i/d(seed) [n_w][6], the signed residual
 * e_i = D_i - r_j of the wire's closest hit (NaN without hits) and whether it is
 * active (|e_i| < lambda). Returns the RSS of Eq. 1 and writes its gradient
 * sum over active wires of 2 e_i J_i to grad[6]. Any output pointer may be NULL. */
static double rss_of_dual_track(const dual *pts, int32_t K, double lambda,
                                const double *wire_ends, int32_t n_wires,
                                const int32_t *offsets, const double *drift, double *D,
                                double *J, double *resid, uint8_t *active, double grad[6])
{
    double rss = 0.0;
    double g[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t i = 0; i < n_wires; ++i) {
        double frame[8];
        oracle_wire_frame(wire_ends + 6 * i, frame);
        dual Dd = dsqrt(dual_dca2(pts, K + 1, frame));
        double e = NAN, eb = INFINITY;
        for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j) {
            double a = fabs(Dd.v - drift[j]);
            if (a < eb) {
                eb = a;
                e = Dd.v - drift[j];
            }
        }
        double d = eb < lambda ? eb : lambda;
        rss = rss + d * d;
        int act = eb < lambda;
        if (act)
            for (int c = 0; c < 6; ++c)
                g[c] += 2.0 * e * Dd.d[c];
        if (D)
            D[i] = Dd.v;
        if (J)
            for (int c = 0; c < 6; ++c)
                J[6 * i + c] = Dd.d[c];
        if (resid)
            resid[i] = e;
        if (active)
            active[i] = (uint8_t)act;
    }
    if (grad)
        for (int c = 0; c < 6; ++c)
            grad[c] = g[c];
    return rss;
}

double oracle_rss_jacobian(const double seed[6], const double cfg[4], int32_t K,
                           const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                           const double *drift, double *D, double *J, double *resid,
                           uint8_t *active, double grad[6])
{
    dual *pts = (dual *)malloc(sizeof(dual) * 3 * (size_t)(K + 1));
    dual_track(seed, cfg[0], cfg[1], cfg[2], K, pts);
    double rss = rss_of_dual_track(pts, K, cfg[3], wire_ends, n_wires, offsets, drift, D, J,
                                   resid, active, grad);
    free(pts);
    return rss;
}

/* ------------------------------------------------------------ Gauss-Newton / LM
 * Refinement of one seed by Levenberg-Marquardt on the active residuals e_i
 * (|e_i| < lambda) with rows J_i: A = sum J_i J_i^T, b = sum J_i e_i; the step solves
 * (A + mu diag(A)) delta = -b by Cholesky; it is accepted when the RSS of Eq. 1
 * decreases (then mu <- mu / 10 and A, b are re-formed), otherwise mu <- 10 mu. A
 * matrix that is not positive definite counts as a rejected step. n_iter steps. */
static void normal_equations(const double seed[6], const double cfg[4], int32_t K,
                             const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                             const double *drift, double A[36], double b[6], double *rss)
{
    double *J = (double *)malloc(sizeof(double) * 6 * (size_t)(n_wires > 0 ? n_wires : 1));
    double *e = (double *)malloc(sizeof(double) * (size_t)(n_wires > 0 ? n_wires : 1));
    uint8_t *act = (uint8_t *)malloc((size_t)(n_wires > 0 ? n_wires : 1));
    *rss = oracle_rss_jacobian(seed, cfg, K, wire_ends, n_wires, offsets, drift, NULL, J, e,
                               act, NULL);
    for (int r = 0; r < 36; ++r)
        A[r] = 0.0;
    for (int r = 0; r < 6; ++r)
        b[r] = 0.0;
    for (int32_t i = 0; i < n_wires; ++i) {
        if (!act[i])
            continue;
        for (int r = 0; r < 6; ++r) {
            b[r] += J[6 * i + r] * e[i];
            for (int c = 0; c < 6; ++c)
                A[6 * r + c] += J[6 * i + r] * J[6 * i + c];
        }
    }
    free(J);
    free(e);
    free(act);
}

/* Solves M x = r for symmetric positive definite M (6x6) by Cholesky; 0 if M is not
 * positive definite. */
static int cholesky_solve6(const double M[36], const double r[6], double x[6])
{
    double L[36] = {0};
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = M[6 * i + j];
            for (int k = 0; k < j; ++k)
                s -= L[6 * i + k] * L[6 * j + k];
            if (i == j) {
                if (!(s > 0.0))
                    return 0;
                L[6 * i + i] = sqrt(s);
            } else {
                L[6 * i + j] = s / L[6 * j + j];
            }
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k)
            s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k)
            s -= L[6 * k + i] * x[k];
        x[i] = s / L[6 * i + i];
    }
    return 1;
}

/* Refines seed[6] in place; returns the final RSS; *accepted counts accepted steps. */
/* The problem the LM loop minimises: the RSS and normal equations at a seed. */
typedef struct {
    const double *cfg;
    int32_t K;
    const double *wire_ends;
    int32_t n_wires;
    const int32_t *offsets;
    const double *drift;
    const void *field; /* NULL: uniform field; else the map (oracle_field) */
    int32_t stepper;   /* in the map: 0 RK4, 1 RKN */
} lm_problem;

static void lm_normal_equations(const lm_problem *pb, const double seed[6], double A[36],
                                double b[6], double *rss);

static double lm_loop(const lm_problem *pb, double seed[6], int32_t n_iter, double mu0,
                      int32_t *accepted)
{
    double A[36], b[6], rss;
    lm_normal_equations(pb, seed, A, b, &rss);
    double mu = mu0;
    int32_t n_acc = 0;
    for (int32_t it = 0; it < n_iter; ++it) {
        double M[36], rhs[6], delta[6];
        for (int r = 0; r < 36; ++r)
            M[r] = A[r];
        for (int r = 0; r < 6; ++r) {
            M[6 * r + r] = A[6 * r + r] + mu * A[6 * r + r];
            rhs[r] = -b[r];
        }
        if (!cholesky_solve6(M, rhs, delta)) {
            mu = mu * 10.0;
            continue;
        }
        double trial[6];
        for (int r = 0; r < 6; ++r)
            trial[r] = seed[r] + delta[r];
        double A2[36], b2[6], rss2;
        lm_normal_equations(pb, trial, A2, b2, &rss2);
        if (rss2 < rss) {
            for (int r = 0; r < 6; ++r) {
                seed[r] = trial[r];
                b[r] = b2[r];
            }
            for (int r = 0; r < 36; ++r)
                A[r] = A2[r];
            rss = rss2;
            mu = mu / 10.0;
            n_acc += 1;
        } else {
            mu = mu * 10.0;
        }
    }
    if (accepted)
        *accepted = n_acc;
    return rss;
}

double oracle_lm_refine(double seed[6], const double cfg[4], int32_t K, const double *wire_ends,
                        int32_t n_wires, const int32_t *offsets, const double *drift,
                        int32_t n_iter, double mu0, int32_t *accepted)
{
    const lm_problem pb = {cfg, K, wire_ends, n_wires, offsets, drift, NULL, 0};
    return lm_loop(&pb, seed, n_iter, mu0, accepted);
}

/* ------------------------------------------------------------ several references
 * Sec. 2.1: several seeds with the lowest RSS become references for the next scan.
 * The k smallest values in increasing order, ties to the lower index, NaN excluded;
 * -1 fills the rest when fewer than k values are not NaN. Plain sort of the pairs. */
typedef struct {
    double v;
    int64_t i;
} oracle_pair;

static int pair_cmp(const void *a, const void *b)
{
    const oracle_pair *x = (const oracle_pair *)a, *y = (const oracle_pair *)b;
    if (x->v < y->v)
        return -1;
    if (x->v > y->v)
        return 1;
    return x->i < y->i ? -1 : (x->i > y->i ? 1 : 0);
}

void oracle_topk(const double *values, int64_t n, int32_t k, int64_t *out)
{
    oracle_pair *p = (oracle_pair *)malloc(sizeof(oracle_pair) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t s = 0; s < n; ++s)
        if (!isnan(values[s])) {
            p[m].v = values[s];
            p[m].i = s;
            ++m;
        }
    qsort(p, (size_t)m, sizeof(oracle_pair), pair_cmp);
    for (int32_t r = 0; r < k; ++r)
        out[r] = r < m ? p[r].i : -1;
    free(p);
}

/* ------------------------------------------------------------ several references
 * Sec. 2.1: several of the lowest-RSS seeds become the reference points of the
 * next, finer scan, and they are chosen sparse enough that the new seed sets around
 * them do not overlap.
 *
 * Candidates: every seed of a group's n_sub grids (grids[u]: same n, S seeds each;
 * candidate index u * S + i). The new seed set around candidate (u, i) is, per axis
 * a, the interval centred on its axis value with the refined half-span
 * 2 half_a / (n_a - 1) (for n_a = 1 the grid's own centre and half-span). Two such
 * boxes overlap when, in every axis, their centres are equal or lie less than the
 * sum of their half-spans apart: fabs(c1 - c2) < 0.999999999 * (h1 + h2). The factor
 * makes boxes that only touch (centres two spacings apart on one grid) count as
 * disjoint whatever the rounding of the centres.
 *
 * Greedy in increasing (rss, candidate index): a candidate is taken when its box
 * overlaps none taken before, until n_ref are taken; NaN is never taken. Per taken
 * reference r: ref_idx[r], ref_rss[r], and new_grids[r] = its grid refined around it
 * (as oracle_refine_grid). Past the last one taken: -1, NaN, and a copy of
 * new_grids[0] (of grids[0] if none was taken). Returns the number taken. */
static void candidate_box(const double grid[14], const int32_t n[4], int64_t i, double c[4],
                          double h[4])
{
    int32_t idx[4];
    int64_t rest = i;
    for (int a = 3; a >= 0; --a) {
        idx[a] = (int32_t)(rest % n[a]);
        rest /= n[a];
    }
    for (int a = 0; a < 4; ++a) {
        if (n[a] > 1) {
            c[a] = oracle_axis_value(grid[6 + a], grid[10 + a], n[a], idx[a]);
            h[a] = (2.0 * grid[10 + a]) / (double)(n[a] - 1);
        } else {
            c[a] = grid[6 + a];
            h[a] = grid[10 + a];
        }
    }
}

static int boxes_overlap(const double c1[4], const double h1[4], const double c2[4],
                         const double h2[4])
{
    for (int a = 0; a < 4; ++a)
        if (!(c1[a] == c2[a] || fabs(c1[a] - c2[a]) < 0.999999999 * (h1[a] + h2[a])))
            return 0;
    return 1;
}

int32_t oracle_sparse_select(const double *grids, const double *rss, int32_t n_sub,
                             const int32_t n[4], int32_t n_ref, int64_t *ref_idx,
                             double *ref_rss, double *new_grids)
{
    const int64_t S = (int64_t)n[0] * n[1] * n[2] * n[3];
    const int64_t total = S * n_sub;
    oracle_pair *p = (oracle_pair *)malloc(sizeof(oracle_pair) * (size_t)(total > 0 ? total : 1));
    double *tc = (double *)malloc(sizeof(double) * 4 * (size_t)(n_ref > 0 ? n_ref : 1));
    double *th = (double *)malloc(sizeof(double) * 4 * (size_t)(n_ref > 0 ? n_ref : 1));
    int64_t m = 0;
    for (int64_t j = 0; j < total; ++j)
        if (!isnan(rss[j])) {
            p[m].v = rss[j];
            p[m].i = j;
            ++m;
        }
    qsort(p, (size_t)m, sizeof(oracle_pair), pair_cmp);
    int32_t taken = 0;
    for (int64_t q = 0; q < m && taken < n_ref; ++q) {
        const int64_t j = p[q].i;
        const double *g = grids + 14 * (j / S);
        double c[4], h[4];
        candidate_box(g, n, j % S, c, h);
        int free_box = 1;
        for (int32_t r = 0; r < taken && free_box; ++r)
            if (boxes_overlap(c, h, tc + 4 * r, th + 4 * r))
                free_box = 0;
        if (!free_box)
            continue;
        memcpy(tc + 4 * taken, c, sizeof c);
        memcpy(th + 4 * taken, h, sizeof h);
        ref_idx[taken] = j;
        ref_rss[taken] = p[q].v;
        memcpy(new_grids + 14 * taken, g, 14 * sizeof(double));
        oracle_refine_grid(new_grids + 14 * taken, n, j % S);
        ++taken;
    }
    for (int32_t r = taken; r < n_ref; ++r) {
        ref_idx[r] = -1;
        ref_rss[r] = NAN;
        memcpy(new_grids + 14 * r, taken > 0 ? new_grids : grids, 14 * sizeof(double));
    }
    free(p);
    free(tc);
    free(th);
    return taken;
}

/* ------------------------------------------------------------ half tracks (Sec. 3.1)
 * Missing-layer veto. A finally selected seed of a half track comes with its half set
 * of classified hits (bit 0 of mask, indexed by the half's hits); a seed whose set
 * leaves some layer without a hit is excluded. The half track starts in front of the
 * first layer and runs out to its outermost classified layer L, so every layer
 * 0..L must hold a classified hit. Returns 1 (vetoed) when one is missing or no hit
 * is classified, 0 when none is missing, -1 when a wire's layer lies outside
 * [0, n_layers). Wire i owns hits [wire_offsets[i] - wire_offsets[0],
 * wire_offsets[i + 1] - wire_offsets[0]) of the mask. */
int32_t oracle_layer_veto(const uint8_t *mask, const int32_t *wire_offsets, int32_t n_wires,
                          const int32_t *wire_layer, int32_t n_layers)
{
    int has[256];
    if (n_layers < 1 || n_layers > 256)
        return -1;
    for (int32_t l = 0; l < n_layers; ++l)
        has[l] = 0;
    for (int32_t i = 0; i < n_wires; ++i) {
        if (wire_layer[i] < 0 || wire_layer[i] >= n_layers)
            return -1;
        for (int32_t j = wire_offsets[i]; j < wire_offsets[i + 1]; ++j)
            if (mask[j - wire_offsets[0]] & 1)
                has[wire_layer[i]] = 1;
    }
    int32_t outer = -1;
    for (int32_t l = 0; l < n_layers; ++l)
        if (has[l])
            outer = l;
    if (outer < 0)
        return 1;
    for (int32_t l = 0; l <= outer; ++l)
        if (!has[l])
            return 1;
    return 0;
}

/* Combinatorial merge of two half sets (Sec. 3.1): every entrance seed i and exit
 * seed j (F each) form a complete set when neither is vetoed (veto == 0) and neither
 * RSS is NaN. With no fit, complete sets are ranked by their combined RSS
 * rss_a[i] + rss_b[j] (each half's RSS over its own wires; the halves share no
 * wire), ascending, ties by the pair index i F + j. pair[k] = i F + j of rank k and
 * pair_rss[k] its combined RSS; -1 and NaN past the last. Returns the number of
 * complete sets. */
typedef struct {
    double v;
    int32_t k;
} oracle_rank;

static int rank_cmp(const void *x, const void *y)
{
    const oracle_rank *a = (const oracle_rank *)x, *b = (const oracle_rank *)y;
    if (a->v < b->v)
        return -1;
    if (a->v > b->v)
        return 1;
    return (a->k > b->k) - (a->k < b->k);
}

int32_t oracle_merge_halves(const double *rss_a, const int32_t *veto_a, const double *rss_b,
                            const int32_t *veto_b, int32_t F, int32_t *pair, double *pair_rss)
{
    oracle_rank *r = (oracle_rank *)malloc(sizeof(oracle_rank) * (size_t)(F > 0 ? F * F : 1));
    int32_t m = 0;
    for (int32_t i = 0; i < F; ++i)
        for (int32_t j = 0; j < F; ++j) {
            if (veto_a[i] != 0 || veto_b[j] != 0 || isnan(rss_a[i]) || isnan(rss_b[j]))
                continue;
            r[m].v = rss_a[i] + rss_b[j];
            r[m].k = i * F + j;
            ++m;
        }
    qsort(r, (size_t)m, sizeof(oracle_rank), rank_cmp);
    for (int32_t k = 0; k < F * F; ++k) {
        pair[k] = k < m ? r[k].k : -1;
        pair_rss[k] = k < m ? r[k].v : NAN;
    }
    free(r);
    return m;
}

/* ------------------------------------------------------------ stage loop (Sec. 3.1)
 * Backward extrapolation to the previous turn partition: the fitted track of a stage
 * is extrapolated backwards to the seed region of the previous turn, which gives the
 * longitudinal seed (z, p_z) of the next stage. From seed6 (x, p) at the current
 * turn's outward crossing of r = radius, the track runs backwards (momentum and
 * charge flipped) with the RK4 step of oracle_track, each step's full state kept.
 * Backwards, the track first heads inwards, comes out again through r = radius (the
 * previous turn's exit) and goes back in through it (the previous turn's entry): the
 * answer is the first inward crossing after an outward one. Between the states a and
 * b of the step that crosses, with d = r^2 - radius^2 (r^2 = x x + y y) >= 0 at a and
 * < 0 at b, f = d_a / (d_a - d_b) and every component is fma(f, b - a, a); the
 * momentum is flipped back. out6 is NaN when no such crossing comes within
 * max_steps. Returns the step count at the crossing (-1 if none). */
int32_t oracle_backward_seed(const double seed6[6], double bz, double charge, double h,
                             double radius, int32_t max_steps, double out6[6])
{
    double s[6] = {seed6[0], seed6[1], seed6[2], -seed6[3], -seed6[4], -seed6[5]};
    const rk4_consts kc = rk4_setup(s[3], s[4], s[5], bz, -charge, h);
    const double R2 = radius * radius;
    int out_seen = 0;
    for (int32_t k = 0; k < 6; ++k)
        out6[k] = NAN;
    for (int32_t k = 1; k <= max_steps; ++k) {
        double a[6];
        for (int j = 0; j < 6; ++j)
            a[j] = s[j];
        rk4_step(&kc, &s[0], &s[1], &s[2], &s[3], &s[4]);
        const double da = (a[0] * a[0] + a[1] * a[1]) - R2;
        const double db = (s[0] * s[0] + s[1] * s[1]) - R2;
        if (da < 0.0 && db >= 0.0)
            out_seen = 1;
        else if (out_seen && da >= 0.0 && db < 0.0) {
            const double f = da / (da - db);
            for (int j = 0; j < 6; ++j)
                out6[j] = fma(f, s[j] - a[j], a[j]);
            out6[3] = -out6[3];
            out6[4] = -out6[4];
            out6[5] = -out6[5];
            return k;
        }
    }
    return -1;
}

/* The exit half track's seed (Sec. 3.1: each turn partition is split into an entrance
 * and an exit half track; the exit half runs backwards from where the turn leaves the
 * seed region). From seed6 at the turn's outward crossing of r = radius, the track runs
 * forwards with the RK4 step of oracle_track until it crosses r = radius inwards after
 * having been outside it: the first step a -> b with d_a >= 0 > d_b (d = x x + y y -
 * radius^2) once some state had d > 0. Every component is fma(f, b - a, a) with
 * f = d_a / (d_a - d_b); then the momentum is reversed (the exit half is scanned with
 * the charge reversed as well). out6 is NaN when no crossing comes within max_steps.
 * Returns the step count at the crossing (-1 if none). */
int32_t oracle_exit_seed(const double seed6[6], double bz, double charge, double h,
                         double radius, int32_t max_steps, double out6[6])
{
    double s[6];
    for (int j = 0; j < 6; ++j)
        s[j] = seed6[j];
    const rk4_consts kc = rk4_setup(s[3], s[4], s[5], bz, charge, h);
    const double R2 = radius * radius;
    int outside = 0;
    for (int32_t k = 0; k < 6; ++k)
        out6[k] = NAN;
    for (int32_t k = 0; k < max_steps; ++k) {
        double a[6];
        for (int j = 0; j < 6; ++j)
            a[j] = s[j];
        rk4_step(&kc, &s[0], &s[1], &s[2], &s[3], &s[4]);
        const double da = (a[0] * a[0] + a[1] * a[1]) - R2;
        const double db = (s[0] * s[0] + s[1] * s[1]) - R2;
        if (da > 0.0)
            outside = 1;
        if (outside && da >= 0.0 && db < 0.0) {
            const double w = da / (da - db);
            for (int j = 0; j < 3; ++j)
                out6[j] = fma(w, s[j] - a[j], a[j]);
            for (int j = 3; j < 6; ++j)
                out6[j] = -fma(w, s[j] - a[j], a[j]);
            return k;
        }
    }
    return -1;
}

/* The next stage's grid descriptor: the transverse seed (x, y, p_x, p_y) of the turn
 * (the Hough-transform seed of Sec. 3.1) with (z, p_z) from the backward
 * extrapolation; axis centres (0, |p|, 0, 0) with |p| = sqrt((px px + py py) + pz pz)
 * and the given half-spans. */
void oracle_stage_grid(const double transverse6[6], const double ext6[6], const double half[4],
                       double grid[14])
{
    for (int j = 0; j < 6; ++j)
        grid[j] = transverse6[j];
    grid[2] = ext6[2];
    grid[5] = ext6[5];
    grid[6] = 0.0;
    grid[7] = sqrt((grid[3] * grid[3] + grid[4] * grid[4]) + grid[5] * grid[5]);
    grid[8] = 0.0;
    grid[9] = 0.0;
    for (int a = 0; a < 4; ++a)
        grid[10 + a] = half[a];
}

/* The seed's z as a fifth grid axis (Sec. 3.1: the seed has five degrees of freedom):
 * grids[u] (u < n_z) is the stage grid with the reference z moved to the u-th of n_z
 * values spread evenly over ext6[2] +- z_half (the rule of the other axes). */
void oracle_stage_grids_z(const double transverse6[6], const double ext6[6],
                          const double half[4], int32_t n_z, double z_half, double *grids)
{
    for (int32_t u = 0; u < n_z; ++u) {
        double *g = grids + 14 * (size_t)u;
        oracle_stage_grid(transverse6, ext6, half, g);
        g[2] = oracle_axis_value(ext6[2], z_half, n_z, u);
    }
}

/* Exclusion of classified hits (Sec. 3.1: hits classified at earlier stages are left
 * out of later scans, so the wire count shrinks). One event in CSR (wire i owns hits
 * [offsets[i], offsets[i+1]), offsets[0] = 0): hits with exclude[j] != 0 are dropped,
 * then wires left without hits; the order of what remains is kept. Writes the new
 * CSR (offsets_out[n_out + 1], drift_out, ends_out[n_out][6]), wire_map[i'] = old wire
 * and hit_map[j'] = old hit; returns n_out. */
int32_t oracle_exclude_hits(int32_t n_wires, const int32_t *offsets, const double *drift,
                            const double *ends, const uint8_t *exclude, int32_t *offsets_out,
                            double *drift_out, double *ends_out, int32_t *wire_map,
                            int32_t *hit_map)
{
    int32_t nw = 0, nh = 0;
    offsets_out[0] = 0;
    for (int32_t i = 0; i < n_wires; ++i) {
        const int32_t h0 = nh;
        for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j)
            if (!exclude[j]) {
                drift_out[nh] = drift[j];
                hit_map[nh] = j;
                ++nh;
            }
        if (nh > h0) {
            for (int c = 0; c < 6; ++c)
                ends_out[6 * nw + c] = ends[6 * i + c];
            wire_map[nw] = i;
            ++nw;
            offsets_out[nw] = nh;
        }
    }
    return nw;
}

/* Self-refining of a stage's classified hits (Sec. 3.1). The paper re-fits the best
 * complete set with the deterministic annealing filter, drops the hits that the fit
 * weights down, and on wires left with hits none of which is classified re-examines
 * those hits against the fitted track with a second cutoff eta. Without that filter
 * the fitted track is the track of seed_fit (the stage's chosen seed after a
 * Levenberg-Marquardt minimisation of Eq. 1), and with D the wire's DCA to it:
 *   (1) a hit classified in mask_in (bit 0) stays classified iff |D - r_j| < lambda;
 *   (2) on a wire where no hit stays classified, the hit with the smallest |D - r_j|
 *       (lowest index on ties) is classified iff that residual is below eta.
 * mask_out[j] = 1 for a classified hit, else 0 (mask_out may be mask_in). A seed
 * with a NaN component (no fit) keeps bit 0 of mask_in. Returns the number of hits
 * classified. */
int32_t oracle_self_refine(const double seed_fit[6], const double cfg[4], int32_t K,
                           const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                           const double *drift, const uint8_t *mask_in, double eta,
                           uint8_t *mask_out)
{
    int fitted = 1;
    for (int c = 0; c < 6; ++c)
        if (isnan(seed_fit[c]))
            fitted = 0;
    int32_t n_cls = 0;
    if (!fitted) {
        for (int32_t j = offsets[0]; j < offsets[n_wires]; ++j) {
            mask_out[j] = mask_in[j] & 1;
            n_cls += mask_out[j];
        }
        return n_cls;
    }
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
    oracle_track(seed_fit, cfg[0], cfg[1], cfg[2], K, pts);
    for (int32_t i = 0; i < n_wires; ++i) {
        double frame[8];
        oracle_wire_frame(wire_ends + 6 * i, frame);
        const double D = sqrt(oracle_dca2(pts, K + 1, frame, NULL));
        int32_t kept = 0;
        for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j) {
            const uint8_t was = mask_in[j] & 1;
            mask_out[j] = (was && fabs(D - drift[j]) < cfg[3]) ? 1 : 0;
            kept += mask_out[j];
        }
        if (kept == 0) {
            int32_t jb = -1;
            double eb = INFINITY;
            for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j) {
                const double e = fabs(D - drift[j]);
                if (e < eb) {
                    eb = e;
                    jb = j;
                }
            }
            if (jb >= 0 && eb < eta) {
                mask_out[jb] = 1;
                kept = 1;
            }
        }
        n_cls += kept;
    }
    free(pts);
    return n_cls;
}

/* ------------------------------------------------------------ field map (Sec. 2.2.1)
 * The paper extrapolates tracks through the solenoid's field map. Here the map is a
 * regular grid of B (tesla) at nodes (x0 + i dx, y0 + j dy, z0 + k dz), i < nx, j < ny,
 * k < nz, stored b[((k ny + j) nx + i) 3 + c]. B at a point: each coordinate u = (x -
 * x0) / dx is clamped to [0, nx - 1], i = min(floor(u), nx - 2), t = u - i, and B is
 * interpolated trilinearly with lerp(a, b, t) = fma(t, b - a, a): first along x (four
 * edges, in the order (j, k) = (0,0), (1,0), (0,1), (1,1)), then along y, then along z. */
typedef struct {
    const double *b;
    int32_t nx, ny, nz;
    double x0, y0, z0, dx, dy, dz;
} oracle_field;

static double lerp(double a, double b, double t) { return fma(t, b - a, a); }

static void cell(double u, int32_t n, int32_t *i, double *t)
{
    if (!(u > 0.0))
        u = 0.0;  /* NaN lands here too */
    if (u > (double)(n - 1))
        u = (double)(n - 1);
    int32_t k = (int32_t)floor(u);
    if (k > n - 2)
        k = n - 2;
    *i = k;
    *t = u - (double)k;
}

static void field_at(const oracle_field *f, double x, double y, double z, double B[3])
{
    int32_t i, j, k;
    double tu, tv, tw;
    cell((x - f->x0) / f->dx, f->nx, &i, &tu);
    cell((y - f->y0) / f->dy, f->ny, &j, &tv);
    cell((z - f->z0) / f->dz, f->nz, &k, &tw);
    for (int c = 0; c < 3; ++c) {
#define NODE(a, b2, c2) f->b[((((int64_t)(k + (c2))) * f->ny + (j + (b2))) * f->nx + (i + (a))) * 3 + c]
        const double c00 = lerp(NODE(0, 0, 0), NODE(1, 0, 0), tu);
        const double c10 = lerp(NODE(0, 1, 0), NODE(1, 1, 0), tu);
        const double c01 = lerp(NODE(0, 0, 1), NODE(1, 0, 1), tu);
        const double c11 = lerp(NODE(0, 1, 1), NODE(1, 1, 1), tu);
#undef NODE
        B[c] = lerp(lerp(c00, c10, tv), lerp(c01, c11, tv), tw);
    }
}

void oracle_field_at(const double *b, const int32_t n[3], const double origin[3],
                     const double step[3], double x, double y, double z, double B[3])
{
    oracle_field f = {b, n[0], n[1], n[2], origin[0], origin[1], origin[2],
                      step[0], step[1], step[2]};
    field_at(&f, x, y, z, B);
}

/* RK4 in a field map. dx/ds = p / p0, dp/ds = ((KAPPA q) / p0) (p x B(x)), p0 = |p| of
 * the seed; every stage evaluates B at its own position:
 *   k1 at (x, p); k2 at (x + h/2 v1, p + h/2 f1); k3 at (x + h/2 v2, p + h/2 f2);
 *   k4 at (x + h v3, p + h f3); y <- y + h/6 (((k1 + 2 k2) + 2 k3) + k4),
 * with v = p inv, f = g (p x B) where g = (KAPPA q) inv, and the cross product
 * (p_y B_z - p_z B_y, p_z B_x - p_x B_z, p_x B_y - p_y B_x). pts: AoS [K+1][3]. */
static void field_force(const oracle_field *fm, double g, const double x[3], const double p[3],
                        double f[3])
{
    double B[3];
    field_at(fm, x[0], x[1], x[2], B);
    f[0] = g * (p[1] * B[2] - p[2] * B[1]);
    f[1] = g * (p[2] * B[0] - p[0] * B[2]);
    f[2] = g * (p[0] * B[1] - p[1] * B[0]);
}

void oracle_track_field(const double seed[6], const double *b, const int32_t n[3],
                        const double origin[3], const double step[3], double charge, double h,
                        int32_t K, double *pts)
{
    oracle_field fm = {b, n[0], n[1], n[2], origin[0], origin[1], origin[2],
                       step[0], step[1], step[2]};
    double x[3] = {seed[0], seed[1], seed[2]}, p[3] = {seed[3], seed[4], seed[5]};
    const double p0 = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const double inv = 1.0 / p0;
    const double g = (ORACLE_KAPPA * charge) * inv;
    const double hh = 0.5 * h, h6 = h / 6.0;
    for (int32_t j = 0; j < K; ++j) {
        for (int c = 0; c < 3; ++c)
            pts[3 * j + c] = x[c];
        double v1[3], f1[3], v2[3], f2[3], v3[3], f3[3], v4[3], f4[3], xs[3], ps[3];
        for (int c = 0; c < 3; ++c)
            v1[c] = p[c] * inv;
        field_force(&fm, g, x, p, f1);
        for (int c = 0; c < 3; ++c) {
            xs[c] = x[c] + hh * v1[c];
            ps[c] = p[c] + hh * f1[c];
            v2[c] = ps[c] * inv;
        }
        field_force(&fm, g, xs, ps, f2);
        for (int c = 0; c < 3; ++c) {
            xs[c] = x[c] + hh * v2[c];
            ps[c] = p[c] + hh * f2[c];
            v3[c] = ps[c] * inv;
        }
        field_force(&fm, g, xs, ps, f3);
        for (int c = 0; c < 3; ++c) {
            xs[c] = x[c] + h * v3[c];
            ps[c] = p[c] + h * f3[c];
            v4[c] = ps[c] * inv;
        }
        field_force(&fm, g, xs, ps, f4);
        for (int c = 0; c < 3; ++c) {
            x[c] = x[c] + h6 * (((v1[c] + 2.0 * v2[c]) + 2.0 * v3[c]) + v4[c]);
            p[c] = p[c] + h6 * (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]);
        }
    }
    for (int c = 0; c < 3; ++c)
        pts[3 * K + c] = x[c];
}

/* Runge-Kutta-Nystrom in a field map (the paper's tracks are extrapolated with RKN):
 * Nystrom's fourth-order method for the second-order equation x'' = a(x, x') in arc
 * length, with the unit direction t = x' (t = p / p0 at the seed) and
 * a(x, t) = g (t x B(x)), g = (KAPPA q) / p0, cross product as in field_force:
 *   a1 = a(x, t)
 *   xm = (x + h/2 t) + h^2/8 a1;  a2 = a(xm, t + h/2 a1);  a3 = a(xm, t + h/2 a2)
 *   xe = (x + h t) + h^2/2 a3;    a4 = a(xe, t + h a3)
 *   x <- (x + h t) + h^2/6 ((a1 + a2) + a3)
 *   t <- t + h/6 (((a1 + 2 a2) + 2 a3) + a4)
 * with hh = 0.5 h, h6 = h / 6, q8 = (h h) / 8, q2 = (h h) * 0.5, q6 = (h h) / 6. a2 and
 * a3 share one read of B at xm: three reads of the map per step instead of RK4's four. */
static void accel(double g, const double t[3], const double B[3], double a[3])
{
    a[0] = g * (t[1] * B[2] - t[2] * B[1]);
    a[1] = g * (t[2] * B[0] - t[0] * B[2]);
    a[2] = g * (t[0] * B[1] - t[1] * B[0]);
}

void oracle_track_field_rkn(const double seed[6], const double *b, const int32_t n[3],
                            const double origin[3], const double step[3], double charge,
                            double h, int32_t K, double *pts)
{
    oracle_field fm = {b, n[0], n[1], n[2], origin[0], origin[1], origin[2],
                       step[0], step[1], step[2]};
    const double p0 = sqrt((seed[3] * seed[3] + seed[4] * seed[4]) + seed[5] * seed[5]);
    const double inv = 1.0 / p0;
    const double g = (ORACLE_KAPPA * charge) * inv;
    const double hh = 0.5 * h, h6 = h / 6.0;
    const double q8 = (h * h) / 8.0, q2 = (h * h) * 0.5, q6 = (h * h) / 6.0;
    double x[3] = {seed[0], seed[1], seed[2]};
    double t[3] = {seed[3] * inv, seed[4] * inv, seed[5] * inv};
    for (int32_t j = 0; j < K; ++j) {
        for (int c = 0; c < 3; ++c)
            pts[3 * j + c] = x[c];
        double B[3], a1[3], a2[3], a3[3], a4[3], xs[3], ts[3];
        field_at(&fm, x[0], x[1], x[2], B);
        accel(g, t, B, a1);
        for (int c = 0; c < 3; ++c) {
            xs[c] = (x[c] + hh * t[c]) + q8 * a1[c];
            ts[c] = t[c] + hh * a1[c];
        }
        field_at(&fm, xs[0], xs[1], xs[2], B);
        accel(g, ts, B, a2);
        for (int c = 0; c < 3; ++c)
            ts[c] = t[c] + hh * a2[c];
        accel(g, ts, B, a3);
        for (int c = 0; c < 3; ++c) {
            xs[c] = (x[c] + h * t[c]) + q2 * a3[c];
            ts[c] = t[c] + h * a3[c];
        }
        field_at(&fm, xs[0], xs[1], xs[2], B);
        accel(g, ts, B, a4);
        for (int c = 0; c < 3; ++c) {
            x[c] = (x[c] + h * t[c]) + q6 * ((a1[c] + a2[c]) + a3[c]);
            t[c] = t[c] + h6 * (((a1[c] + 2.0 * a2[c]) + 2.0 * a3[c]) + a4[c]);
        }
    }
    for (int c = 0; c < 3; ++c)
        pts[3 * K + c] = x[c];
}

/* Derivatives in a field map: the same per-wire outputs as oracle_rss_jacobian for the
 * track of oracle_track_field, in dual numbers. B(x) enters the chain through the
 * trilinear interpolation: the fractions t of a cell are duals, so each stage's force
 * carries dB/dx (piecewise constant in each cell's t, as the interpolation is); a
 * coordinate clamped to the grid is a constant there, as the plain function's value is.
 * The values are computed with the operations of oracle_track_field. */
static dual dual_lerp(dual a, dual b, dual t) { return dfma(t, dsub(b, a), a); }

static void dual_cell(dual u, int32_t n, int32_t *i, dual *t)
{
    if (!(u.v > 0.0))
        u = dc(0.0);
    if (u.v > (double)(n - 1))
        u = dc((double)(n - 1));
    int32_t k = (int32_t)floor(u.v);
    if (k > n - 2)
        k = n - 2;
    *i = k;
    *t = dsub(u, dc((double)k));
}

static void dual_field_at(const oracle_field *f, const dual x[3], dual B[3])
{
    int32_t i, j, k;
    dual tu, tv, tw;
    dual_cell(ddiv(dsub(x[0], dc(f->x0)), dc(f->dx)), f->nx, &i, &tu);
    dual_cell(ddiv(dsub(x[1], dc(f->y0)), dc(f->dy)), f->ny, &j, &tv);
    dual_cell(ddiv(dsub(x[2], dc(f->z0)), dc(f->dz)), f->nz, &k, &tw);
    for (int c = 0; c < 3; ++c) {
#define NODE(a, b2, c2) dc(f->b[((((int64_t)(k + (c2))) * f->ny + (j + (b2))) * f->nx + (i + (a))) * 3 + c])
        const dual c00 = dual_lerp(NODE(0, 0, 0), NODE(1, 0, 0), tu);
        const dual c10 = dual_lerp(NODE(0, 1, 0), NODE(1, 1, 0), tu);
        const dual c01 = dual_lerp(NODE(0, 0, 1), NODE(1, 0, 1), tu);
        const dual c11 = dual_lerp(NODE(0, 1, 1), NODE(1, 1, 1), tu);
#undef NODE
        B[c] = dual_lerp(dual_lerp(c00, c10, tv), dual_lerp(c01, c11, tv), tw);
    }
}

static void dual_field_force(const oracle_field *fm, dual g, const dual x[3], const dual p[3],
                             dual f[3])
{
    dual B[3];
    dual_field_at(fm, x, B);
    f[0] = dmul(g, dsub(dmul(p[1], B[2]), dmul(p[2], B[1])));
    f[1] = dmul(g, dsub(dmul(p[2], B[0]), dmul(p[0], B[2])));
    f[2] = dmul(g, dsub(dmul(p[0], B[1]), dmul(p[1], B[0])));
}

static void dual_track_field(const double seed[6], const oracle_field *fm, double charge,
                             double h, int32_t K, dual *pts)
{
    dual x[3] = {dvar(seed[0], 0), dvar(seed[1], 1), dvar(seed[2], 2)};
    dual p[3] = {dvar(seed[3], 3), dvar(seed[4], 4), dvar(seed[5], 5)};
    const dual p0 = dsqrt(dadd(dadd(dmul(p[0], p[0]), dmul(p[1], p[1])), dmul(p[2], p[2])));
    const dual inv = ddiv(dc(1.0), p0);
    const dual g = dmul(dc(ORACLE_KAPPA * charge), inv);
    const dual hh = dc(0.5 * h), hd = dc(h), h6 = dc(h / 6.0), two = dc(2.0);
    for (int32_t j = 0; j < K; ++j) {
        for (int c = 0; c < 3; ++c)
            pts[3 * j + c] = x[c];
        dual v1[3], f1[3], v2[3], f2[3], v3[3], f3[3], v4[3], f4[3], xs[3], ps[3];
        for (int c = 0; c < 3; ++c)
            v1[c] = dmul(p[c], inv);
        dual_field_force(fm, g, x, p, f1);
        for (int c = 0; c < 3; ++c) {
            xs[c] = dadd(x[c], dmul(hh, v1[c]));
            ps[c] = dadd(p[c], dmul(hh, f1[c]));
            v2[c] = dmul(ps[c], inv);
        }
        dual_field_force(fm, g, xs, ps, f2);
        for (int c = 0; c < 3; ++c) {
            xs[c] = dadd(x[c], dmul(hh, v2[c]));
            ps[c] = dadd(p[c], dmul(hh, f2[c]));
            v3[c] = dmul(ps[c], inv);
        }
        dual_field_force(fm, g, xs, ps, f3);
        for (int c = 0; c < 3; ++c) {
            xs[c] = dadd(x[c], dmul(hd, v3[c]));
            ps[c] = dadd(p[c], dmul(hd, f3[c]));
            v4[c] = dmul(ps[c], inv);
        }
        dual_field_force(fm, g, xs, ps, f4);
        for (int c = 0; c < 3; ++c) {
            x[c] = dadd(x[c], dmul(h6, dadd(dadd(dadd(v1[c], dmul(two, v2[c])), dmul(two, v3[c])),
                                            v4[c])));
            p[c] = dadd(p[c], dmul(h6, dadd(dadd(dadd(f1[c], dmul(two, f2[c])), dmul(two, f3[c])),
                                            f4[c])));
        }
    }
    for (int c = 0; c < 3; ++c)
        pts[3 * K + c] = x[c];
}

/* oracle_track_field_rkn in dual numbers (B and dB/dx shared by a2 and a3 as there). */
static void dual_accel(dual g, const dual t[3], const dual B[3], dual a[3])
{
    a[0] = dmul(g, dsub(dmul(t[1], B[2]), dmul(t[2], B[1])));
    a[1] = dmul(g, dsub(dmul(t[2], B[0]), dmul(t[0], B[2])));
    a[2] = dmul(g, dsub(dmul(t[0], B[1]), dmul(t[1], B[0])));
}

static void dual_track_field_rkn(const double seed[6], const oracle_field *fm, double charge,
                                 double h, int32_t K, dual *pts)
{
    dual x[3] = {dvar(seed[0], 0), dvar(seed[1], 1), dvar(seed[2], 2)};
    dual p[3] = {dvar(seed[3], 3), dvar(seed[4], 4), dvar(seed[5], 5)};
    const dual p0 = dsqrt(dadd(dadd(dmul(p[0], p[0]), dmul(p[1], p[1])), dmul(p[2], p[2])));
    const dual inv = ddiv(dc(1.0), p0);
    const dual g = dmul(dc(ORACLE_KAPPA * charge), inv);
    const dual hh = dc(0.5 * h), hd = dc(h), h6 = dc(h / 6.0), two = dc(2.0);
    const dual q8 = dc((h * h) / 8.0), q2 = dc((h * h) * 0.5), q6 = dc((h * h) / 6.0);
    dual t[3] = {dmul(p[0], inv), dmul(p[1], inv), dmul(p[2], inv)};
    for (int32_t j = 0; j < K; ++j) {
        for (int c = 0; c < 3; ++c)
            pts[3 * j + c] = x[c];
        dual B[3], a1[3], a2[3], a3[3], a4[3], xs[3], ts[3];
        dual_field_at(fm, x, B);
        dual_accel(g, t, B, a1);
        for (int c = 0; c < 3; ++c) {
            xs[c] = dadd(dadd(x[c], dmul(hh, t[c])), dmul(q8, a1[c]));
            ts[c] = dadd(t[c], dmul(hh, a1[c]));
        }
        dual_field_at(fm, xs, B);
        dual_accel(g, ts, B, a2);
        for (int c = 0; c < 3; ++c)
            ts[c] = dadd(t[c], dmul(hh, a2[c]));
        dual_accel(g, ts, B, a3);
        for (int c = 0; c < 3; ++c) {
            xs[c] = dadd(dadd(x[c], dmul(hd, t[c])), dmul(q2, a3[c]));
            ts[c] = dadd(t[c], dmul(hd, a3[c]));
        }
        dual_field_at(fm, xs, B);
        dual_accel(g, ts, B, a4);
        for (int c = 0; c < 3; ++c) {
            x[c] = dadd(dadd(x[c], dmul(hd, t[c])), dmul(q6, dadd(dadd(a1[c], a2[c]), a3[c])));
            t[c] = dadd(t[c], dmul(h6, dadd(dadd(dadd(a1[c], dmul(two, a2[c])), dmul(two, a3[c])),
                                            a4[c])));
        }
    }
    for (int c = 0; c < 3; ++c)
        pts[3 * K + c] = x[c];
}

/* stepper: 0 = RK4 (oracle_track_field), 1 = RKN (oracle_track_field_rkn). */
double oracle_rss_jacobian_field(const double seed[6], const double *b, const int32_t n[3],
                                 const double origin[3], const double step[3], double charge,
                                 double h, int32_t K, double lambda, const double *wire_ends,
                                 int32_t n_wires, const int32_t *offsets, const double *drift,
                                 double *D, double *J, double *resid, uint8_t *active,
                                 double grad[6], int32_t stepper)
{
    oracle_field fm = {b, n[0], n[1], n[2], origin[0], origin[1], origin[2],
                       step[0], step[1], step[2]};
    dual *pts = (dual *)malloc(sizeof(dual) * 3 * (size_t)(K + 1));
    if (stepper == 1)
        dual_track_field_rkn(seed, &fm, charge, h, K, pts);
    else
        dual_track_field(seed, &fm, charge, h, K, pts);
    double rss = rss_of_dual_track(pts, K, lambda, wire_ends, n_wires, offsets, drift, D, J,
                                   resid, active, grad);
    free(pts);
    return rss;
}

/* Levenberg-Marquardt in a field map: oracle_lm_refine with the derivatives and RSS of
 * the map's tracks (oracle_rss_jacobian_field). */
static void lm_normal_equations(const lm_problem *pb, const double seed[6], double A[36],
                                double b[6], double *rss)
{
    if (!pb->field) {
        normal_equations(seed, pb->cfg, pb->K, pb->wire_ends, pb->n_wires, pb->offsets,
                         pb->drift, A, b, rss);
        return;
    }
    const oracle_field *f = (const oracle_field *)pb->field;
    const int32_t n_w = pb->n_wires;
    double *J = (double *)malloc(sizeof(double) * 6 * (size_t)(n_w > 0 ? n_w : 1));
    double *e = (double *)malloc(sizeof(double) * (size_t)(n_w > 0 ? n_w : 1));
    uint8_t *act = (uint8_t *)malloc((size_t)(n_w > 0 ? n_w : 1));
    const int32_t n[3] = {f->nx, f->ny, f->nz};
    const double origin[3] = {f->x0, f->y0, f->z0}, step[3] = {f->dx, f->dy, f->dz};
    *rss = oracle_rss_jacobian_field(seed, f->b, n, origin, step, pb->cfg[1], pb->cfg[2], pb->K,
                                     pb->cfg[3], pb->wire_ends, n_w, pb->offsets, pb->drift,
                                     NULL, J, e, act, NULL, pb->stepper);
    for (int r = 0; r < 36; ++r)
        A[r] = 0.0;
    for (int r = 0; r < 6; ++r)
        b[r] = 0.0;
    for (int32_t i = 0; i < n_w; ++i) {
        if (!act[i])
            continue;
        for (int r = 0; r < 6; ++r) {
            b[r] += J[6 * i + r] * e[i];
            for (int c = 0; c < 6; ++c)
                A[6 * r + c] += J[6 * i + r] * J[6 * i + c];
        }
    }
    free(J);
    free(e);
    free(act);
}

double oracle_lm_refine_field(double seed[6], const double *b, const int32_t n[3],
                              const double origin[3], const double step[3], const double cfg[4],
                              int32_t K, const double *wire_ends, int32_t n_wires,
                              const int32_t *offsets, const double *drift, int32_t n_iter,
                              double mu0, int32_t *accepted, int32_t stepper)
{
    const oracle_field fm = {b, n[0], n[1], n[2], origin[0], origin[1], origin[2],
                             step[0], step[1], step[2]};
    const lm_problem pb = {cfg, K, wire_ends, n_wires, offsets, drift, &fm, stepper};
    return lm_loop(&pb, seed, n_iter, mu0, accepted);
}

/* The whole path for one turn partition (oracle_scan_partition's steps: grid scan,
 * n_refine finer re-scans, classification at the final best) with every track in a
 * field map, RK4 (stepper 0, oracle_track_field) or RKN (1, oracle_track_field_rkn);
 * cfg = (unused, charge, h, lambda). Single-threaded. */
int64_t oracle_scan_partition_field(double grid[14], const int32_t n[4], const double *b,
                                    const int32_t nmap[3], const double origin[3],
                                    const double step[3], int32_t stepper, const double cfg[4],
                                    int32_t K, int32_t n_refine, const double *wire_ends,
                                    int32_t n_wires, const int32_t *offsets, const double *drift,
                                    double *rss_out, double *best_seed, double *best_rss,
                                    uint8_t *mask, int32_t *n_border)
{
    const int64_t S = (int64_t)n[0] * n[1] * n[2] * n[3];
    double *seeds = (double *)malloc(sizeof(double) * 6 * (size_t)S);
    double *rss = rss_out ? rss_out : (double *)malloc(sizeof(double) * (size_t)S);
    double *frames = (double *)malloc(sizeof(double) * 8 * (size_t)(n_wires > 0 ? n_wires : 1));
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
    for (int32_t i = 0; i < n_wires; ++i)
        oracle_wire_frame(wire_ends + 6 * i, frames + 8 * i);
    int64_t best = -1;
    for (int32_t it = 0; it <= n_refine; ++it) {
        if (it > 0)
            oracle_refine_grid(grid, n, best);
        oracle_seed_grid(grid, n, seeds);
        for (int64_t s = 0; s < S; ++s) {
            double seed[6];
            for (int c = 0; c < 6; ++c)
                seed[c] = seeds[c * S + s];
            if (stepper == 1)
                oracle_track_field_rkn(seed, b, nmap, origin, step, cfg[1], cfg[2], K, pts);
            else
                oracle_track_field(seed, b, nmap, origin, step, cfg[1], cfg[2], K, pts);
            rss[s] = oracle_rss_track(pts, K + 1, frames, n_wires, offsets, drift, cfg[3]);
        }
        best = oracle_argmin(rss, S);
    }
    if (best >= 0) {
        oracle_seed(grid, n, best, best_seed);
        *best_rss = rss[best];
        if (stepper == 1)
            oracle_track_field_rkn(best_seed, b, nmap, origin, step, cfg[1], cfg[2], K, pts);
        else
            oracle_track_field(best_seed, b, nmap, origin, step, cfg[1], cfg[2], K, pts);
        const int32_t nb = classify_track(pts, K, cfg, wire_ends, n_wires, offsets, drift, mask,
                                          NULL);
        if (n_border)
            *n_border = nb;
    }
    free(pts);
    free(frames);
    free(seeds);
    if (!rss_out)
        free(rss);
    return best;
}
