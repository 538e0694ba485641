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
void oracle_track(const double seed[6], double bz, double charge, double h, int32_t K,
                  double *pts)
{
    double x = seed[0], y = seed[1], z = seed[2];
    double px = seed[3], py = seed[4], pz = seed[5];
    double p0 = sqrt((px * px + py * py) + pz * pz);
    double inv = 1.0 / p0;
    double c = ((ORACLE_KAPPA * charge) * bz) * inv;
    double hh = 0.5 * h;
    double h6 = h / 6.0;
    double vz = pz * inv; /* z velocity: the same at every stage */

    for (int32_t k = 0; k < K; ++k) {
        pts[3 * k + 0] = x;
        pts[3 * k + 1] = y;
        pts[3 * k + 2] = z;
        /* stage 1 at p */
        double v1x = px * inv, v1y = py * inv;
        double f1x = c * py, f1y = -(c * px);
        /* stage 2 at p + h/2 f1 */
        double qx = px + hh * f1x, qy = py + hh * f1y;
        double v2x = qx * inv, v2y = qy * inv;
        double f2x = c * qy, f2y = -(c * qx);
        /* stage 3 at p + h/2 f2 */
        qx = px + hh * f2x;
        qy = py + hh * f2y;
        double v3x = qx * inv, v3y = qy * inv;
        double f3x = c * qy, f3y = -(c * qx);
        /* stage 4 at p + h f3 */
        qx = px + h * f3x;
        qy = py + h * f3y;
        double v4x = qx * inv, v4y = qy * inv;
        double f4x = c * qy, f4y = -(c * qx);

        x = x + h6 * (((v1x + 2.0 * v2x) + 2.0 * v3x) + v4x);
        y = y + h6 * (((v1y + 2.0 * v2y) + 2.0 * v3y) + v4y);
        z = z + h6 * (((vz + 2.0 * vz) + 2.0 * vz) + vz);
        px = px + h6 * (((f1x + 2.0 * f2x) + 2.0 * f3x) + f4x);
        py = py + h6 * (((f1y + 2.0 * f2y) + 2.0 * f3y) + f4y);
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
int32_t oracle_classify(const double seed[6], const double cfg[4], int32_t K,
                        const double *wire_ends, int32_t n_wires, const int32_t *offsets,
                        const double *drift, uint8_t *mask, double *dca)
{
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
    oracle_track(seed, cfg[0], cfg[1], cfg[2], K, pts);
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
