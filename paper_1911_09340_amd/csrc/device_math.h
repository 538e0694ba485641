// device_math.h -- the evaluation-order contract of the seed-scan path, as device
// functions shared by every kernel of the library (GPU side only).
//
// Paper: Yeo, Lee and Kuno, "GPU-accelerated event reconstruction for the COMET
// Phase-I experiment" (arXiv:1911.09340), Sec. 2 (Alg. 1-3, Eq. 1).
//
// Every formula is evaluated exactly as written: the library is compiled with
// -ffp-contract=off, fma() appears only where written, and division and square
// root are the correctly rounded binary64 operations.
#ifndef COMET_DEVICE_MATH_H
#define COMET_DEVICE_MATH_H

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

namespace cdev {

constexpr double kKappa = 0.299792458;  // MeV/c per (T mm)

// ------------------------------------------------------------------ seed grid
// Axis value i of n: centre (n == 1) or centre + half ((2i - (n-1)) / (n-1)).
__device__ __forceinline__ double axis_value(double centre, double half, int n, int i)
{
    if (n == 1)
        return centre;
    return centre + half * ((double)(2 * i - (n - 1)) / (double)(n - 1));
}

// Rotation by 2 atan(tau): cos = (1 - tau^2) / (1 + tau^2), sin = (2 tau) / (1 + tau^2).
__device__ __forceinline__ void half_angle_rotation(double tau, double &c, double &s)
{
    const double t2 = tau * tau;
    const double den = 1.0 + t2;
    c = (1.0 - t2) / den;
    s = (2.0 * tau) / den;
}

// Seed `index` of a grid descriptor g = (reference state [6], centres [4], half-spans
// [4]) with n0..n3 points per axis (axis 3 fastest). Offsets enter as rotations by
// 2 atan(tau): tau = v0 / (2 r0) on the seed circle, tau = v / 2 for the angles.
__device__ __forceinline__ void seed_from_grid(const double *__restrict__ g, int n0, int n1,
                                               int n2, int n3, int64_t index, double out[6])
{
    const int i3 = (int)(index % n3);
    int64_t rest = index / n3;
    const int i2 = (int)(rest % n2);
    rest /= n2;
    const int i1 = (int)(rest % n1);
    const int i0 = (int)(rest / n1);
    const double v0 = axis_value(g[6], g[10], n0, i0);
    const double v1 = axis_value(g[7], g[11], n1, i1);
    const double v2 = axis_value(g[8], g[12], n2, i2);
    const double v3 = axis_value(g[9], g[13], n3, i3);
    const double x0 = g[0], y0 = g[1], z0 = g[2];
    const double px0 = g[3], py0 = g[4], pz0 = g[5];
    const double r0 = sqrt(x0 * x0 + y0 * y0);
    double ca, sa;
    half_angle_rotation(v0 / (2.0 * r0), ca, sa);
    const double pt0 = sqrt(px0 * px0 + py0 * py0);
    const double p0 = sqrt((px0 * px0 + py0 * py0) + pz0 * pz0);
    const double ct0 = pz0 / p0, st0 = pt0 / p0;
    const double cp0 = px0 / pt0, sp0 = py0 / pt0;
    double cdt, sdt, cdp, sdp;
    half_angle_rotation(v2 * 0.5, cdt, sdt);
    half_angle_rotation(v3 * 0.5, cdp, sdp);
    const double ct = ct0 * cdt - st0 * sdt;
    const double st = st0 * cdt + ct0 * sdt;
    const double cp = cp0 * cdp - sp0 * sdp;
    const double sp = sp0 * cdp + cp0 * sdp;
    out[0] = x0 * ca - y0 * sa;
    out[1] = y0 * ca + x0 * sa;
    out[2] = z0;
    out[3] = v1 * (st * cp);
    out[4] = v1 * (st * sp);
    out[5] = v1 * ct;
}

// Finer re-scan around seed b (Sec. 2.1): each axis with n > 1 is re-centred on b's
// value and its half-span becomes one spacing, (2 half) / (n - 1). b < 0: no change.
__device__ __forceinline__ void refine_grid_desc(double *__restrict__ g, int n0, int n1, int n2,
                                                 int n3, int64_t b)
{
    if (b < 0)
        return;
    const int n[4] = {n0, n1, n2, n3};
    int idx[4];
    int64_t rest = b;
    for (int a = 3; a >= 0; --a) {
        idx[a] = (int)(rest % n[a]);
        rest /= n[a];
    }
    for (int a = 0; a < 4; ++a) {
        if (n[a] > 1) {
            const double v = axis_value(g[6 + a], g[10 + a], n[a], idx[a]);
            g[6 + a] = v;
            g[10 + a] = (2.0 * g[10 + a]) / (double)(n[a] - 1);
        }
    }
}

// ------------------------------------------------------------------ selection
// (value, index) pairs; index < 0 means "nothing yet". a beats b when b is empty,
// or a.v < b.v, or a.v == b.v and a.i < b.i. NaN is never stored.
struct MinLoc {
    double v;
    int64_t i;
};

__device__ __forceinline__ bool beats(const MinLoc &a, const MinLoc &b)
{
    if (a.i < 0)
        return false;
    if (b.i < 0)
        return true;
    return a.v < b.v || (a.v == b.v && a.i < b.i);
}

constexpr int kSelectThreads = 1024;

// First index of the smallest of rss[0..S) (NaN never chosen, -1 if all are NaN), by
// a block of NT threads (a multiple of 64, at most 4096); the result is valid in
// thread 0. Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ int64_t block_argmin_n(const double *__restrict__ rss, int64_t S)
{
    static_assert(NT % 64 == 0 && NT <= 4096, "block size");
    __shared__ double sv[NT / 64];
    __shared__ int64_t si[NT / 64];
    MinLoc m{INFINITY, -1};
    for (int64_t s = threadIdx.x; s < S; s += NT) {
        const double v = rss[s];
        if (v < m.v || (m.i < 0 && v == m.v)) {
            m.v = v;
            m.i = s;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        MinLoc o{__shfl_xor(m.v, off), __shfl_xor(m.i, off)};
        if (beats(o, m))
            m = o;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sv[wave] = m.v;
        si[wave] = m.i;
    }
    __syncthreads();
    MinLoc a{INFINITY, -1};
    if (wave == 0) {
        if (lane < NT / 64) {
            a.v = sv[lane];
            a.i = si[lane];
        }
        for (int off = 32; off > 0; off >>= 1) {
            MinLoc o{__shfl_xor(a.v, off), __shfl_xor(a.i, off)};
            if (beats(o, a))
                a = o;
        }
    }
    return a.i;
}

// The same selection by one wave on its own (no LDS, no barrier): every lane of the
// wave returns the result.
__device__ __forceinline__ int64_t wave_argmin(const double *__restrict__ rss, int64_t S)
{
    MinLoc m{INFINITY, -1};
    for (int64_t s = threadIdx.x & 63; s < S; s += 64) {
        const double v = rss[s];
        if (v < m.v || (m.i < 0 && v == m.v)) {
            m.v = v;
            m.i = s;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        MinLoc o{__shfl_xor(m.v, off), __shfl_xor(m.i, off)};
        if (beats(o, m))
            m = o;
    }
    return m.i;
}

__device__ __forceinline__ int64_t block_argmin(const double *__restrict__ rss, int64_t S)
{
    return block_argmin_n<kSelectThreads>(rss, S);
}

// ------------------------------------------------------------------ RK4 step
// Alg. 1's stepping. ODE in path length: dx/ds = p / p0, dp/ds = c (p_y, -p_x, 0)
// with inv = 1 / p0 and c = ((kappa q) B_z) * inv (uniform field along z; p_z and the
// z velocity vz = p_z * inv never change). One classical RK4 step of length h
// (hh = 0.5 h, h6 = h / 6):
//   v1 = p inv, f1 = c (p_y, -p_x); q = p + hh f1: v2, f2; q = p + hh f2: v3, f3;
//   q = p + h f3: v4, f4; x += h6 (((v1 + 2 v2) + 2 v3) + v4) (y likewise),
//   z += h6 (((vz + 2 vz) + 2 vz) + vz), p += h6 (((f1 + 2 f2) + 2 f3) + f4).
struct StepConsts {
    double inv, c, h, hh, h6, vz;
};

__device__ __forceinline__ StepConsts step_consts(double px, double py, double pz, double bz,
                                                  double charge, double h)
{
    StepConsts k;
    const double p0 = sqrt((px * px + py * py) + pz * pz);
    k.inv = 1.0 / p0;
    k.c = ((kKappa * charge) * bz) * k.inv;
    k.h = h;
    k.hh = 0.5 * h;
    k.h6 = h / 6.0;
    k.vz = pz * k.inv;
    return k;
}

__device__ __forceinline__ void rk4_step(const StepConsts &k, double &x, double &y, double &z,
                                         double &px, double &py)
{
    const double v1x = px * k.inv, v1y = py * k.inv;
    const double f1x = k.c * py, f1y = -(k.c * px);
    double qx = px + k.hh * f1x, qy = py + k.hh * f1y;
    const double v2x = qx * k.inv, v2y = qy * k.inv;
    const double f2x = k.c * qy, f2y = -(k.c * qx);
    qx = px + k.hh * f2x;
    qy = py + k.hh * f2y;
    const double v3x = qx * k.inv, v3y = qy * k.inv;
    const double f3x = k.c * qy, f3y = -(k.c * qx);
    qx = px + k.h * f3x;
    qy = py + k.h * f3y;
    const double v4x = qx * k.inv, v4y = qy * k.inv;
    const double f4x = k.c * qy, f4y = -(k.c * qx);
    x = x + k.h6 * (((v1x + 2.0 * v2x) + 2.0 * v3x) + v4x);
    y = y + k.h6 * (((v1y + 2.0 * v2y) + 2.0 * v3y) + v4y);
    z = z + k.h6 * (((k.vz + 2.0 * k.vz) + 2.0 * k.vz) + k.vz);
    px = px + k.h6 * (((f1x + 2.0 * f2x) + 2.0 * f3x) + f4x);
    py = py + k.h6 * (((f1y + 2.0 * f2y) + 2.0 * f3y) + f4y);
}

// ------------------------------------------------------------------ wire frames
// The distance of a point to a wire is the length of its offset from the wire
// projected on the plane normal to the unit direction n; (e1, e2) spans that plane
// (branch-free orthonormal basis of Duff et al., JCGT 2017):
//   s = copysign(1, n_z), a = -1 / (s + n_z), b = (n_x n_y) a,
//   e1 = (1 + ((s n_x) n_x) a, s b, -(s n_x)),  e2 = (b, s + (n_y n_y) a, -n_y),
//   nc = -((e_x A_x + e_y A_y) + e_z A_z) for endpoint A.
// frame = (e1x, e1y, e1z, nc1, e2x, e2y, e2z, nc2).
__device__ __forceinline__ void wire_frame(const double *__restrict__ ends, double f[8])
{
    const double ax = ends[0], ay = ends[1], az = ends[2];
    const double dx = ends[3] - ax, dy = ends[4] - ay, dz = ends[5] - az;
    const double len = sqrt((dx * dx + dy * dy) + dz * dz);
    const double nx = dx / len, ny = dy / len, nz = dz / len;
    const double s = copysign(1.0, nz);
    const double a = -1.0 / (s + nz);
    const double b = (nx * ny) * a;
    const double e1x = 1.0 + ((s * nx) * nx) * a, e1y = s * b, e1z = -(s * nx);
    const double e2x = b, e2y = s + (ny * ny) * a, e2z = -ny;
    f[0] = e1x;
    f[1] = e1y;
    f[2] = e1z;
    f[3] = -((e1x * ax + e1y * ay) + e1z * az);
    f[4] = e2x;
    f[5] = e2y;
    f[6] = e2z;
    f[7] = -((e2x * ax + e2y * ay) + e2z * az);
}

// In-plane coordinates: xi = fma(e1x, x, fma(e1y, y, fma(e1z, z, nc1))), eta likewise.
__device__ __forceinline__ void project(const double f[8], double x, double y, double z,
                                        double &xi, double &eta)
{
    xi = fma(f[0], x, fma(f[1], y, fma(f[2], z, f[3])));
    eta = fma(f[4], x, fma(f[5], y, fma(f[6], z, f[7])));
}

// Squared distance from the wire to the chord a -> b (in-plane coordinates):
// u = b - a, g = fma(a_xi, u_xi, a_eta u_eta), den = fma(u_xi, u_xi, u_eta u_eta);
// t = 0 (g >= 0) gives qa, t = 1 (-g >= den) gives qb, otherwise t = -g / den and
// the point a + t u gives fma(p_xi, p_xi, p_eta p_eta).
__device__ __forceinline__ double chord_distance2(double axi, double aeta, double qa, double bxi,
                                                  double beta, double qb)
{
    const double uxi = bxi - axi, ueta = beta - aeta;
    const double g = fma(axi, uxi, aeta * ueta);
    const double den = fma(uxi, uxi, ueta * ueta);
    if (!(g < 0.0))
        return qa;
    if (-g >= den)
        return qb;
    const double t = -g / den;
    const double pxi = fma(t, uxi, axi), peta = fma(t, ueta, aeta);
    return fma(pxi, pxi, peta * peta);
}

// Alg. 2's local refinement from the closest recorded point k (value qk): the
// squared DCA is min(qk, chord(k-1 -> k), chord(k -> k+1)). Point j is
// (tx[j ld], ty[j ld], tz[j ld]).
__device__ __forceinline__ double refine_dca2(const double *__restrict__ tx,
                                              const double *__restrict__ ty,
                                              const double *__restrict__ tz, int64_t ld, int P,
                                              const double f[8], int k, double qk)
{
    double cxi, ceta;
    const int64_t oc = (int64_t)k * ld;
    project(f, tx[oc], ty[oc], tz[oc], cxi, ceta);
    double d2 = qk;
    if (k > 0) {
        const int64_t o = (int64_t)(k - 1) * ld;
        double xi, eta;
        project(f, tx[o], ty[o], tz[o], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(xi, eta, q, cxi, ceta, qk);
        if (v < d2)
            d2 = v;
    }
    if (k < P - 1) {
        const int64_t o = (int64_t)(k + 1) * ld;
        double xi, eta;
        project(f, tx[o], ty[o], tz[o], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(cxi, ceta, qk, xi, eta, q);
        if (v < d2)
            d2 = v;
    }
    return d2;
}

// The same with the three points already loaded (pm: point k - 1, read only when k > 0;
// pc: point k; pn: point k + 1, read only when k < P - 1): the same arithmetic in the
// same order, for callers that load the points of several wires before refining any.
__device__ __forceinline__ double refine_dca2_at(const double f[8], int k, int P, double qk,
                                                 const double (&pm)[3], const double (&pc)[3],
                                                 const double (&pn)[3])
{
    double cxi, ceta;
    project(f, pc[0], pc[1], pc[2], cxi, ceta);
    double d2 = qk;
    if (k > 0) {
        double xi, eta;
        project(f, pm[0], pm[1], pm[2], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(xi, eta, q, cxi, ceta, qk);
        if (v < d2)
            d2 = v;
    }
    if (k < P - 1) {
        double xi, eta;
        project(f, pn[0], pn[1], pn[2], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(cxi, ceta, qk, xi, eta, q);
        if (v < d2)
            d2 = v;
    }
    return d2;
}

// The same with the seed-fastest track layout [3][P][S]: point j of seed s is
// track[(c P + j) S + s].
__device__ __forceinline__ double refine_dca2(const double *__restrict__ track, int64_t S, int P,
                                              int64_t s, const double f[8], int k, double qk)
{
    const int64_t PS = (int64_t)P * S;
    return refine_dca2(track + s, track + PS + s, track + 2 * PS + s, S, P, f, k, qk);
}

// Chunk radii of a recorded track, for the distance bound of the DCA scan. Window n
// holds points 16 n ... min(16 n + 16, P - 1) (consecutive windows share their end
// point) and rho[n] = max |p_k - p_(16 n)| over it, so that a 32-point chunk starting
// at 16 n lies within rho[n] + rho[n + 1] of its first point. Feed every point in
// order; NaN distances are ignored (a NaN first point makes the bound unused: its q
// is NaN and the scan never skips such a chunk). Row radius_chunks(P) receives the
// longest step |p_(k+1) - p_k| of the track (+inf when a step is NaN), which bounds
// the length of every chord (the wide scan's cap, TileScanWide).
constexpr int kRadiusChunk = 16;

__host__ __device__ constexpr int radius_chunks(int P) { return (P - 1) / kRadiusChunk + 1; }
// rows of a track's radius array: the windows, then the longest step
__host__ __device__ constexpr int radius_rows(int P) { return radius_chunks(P) + 1; }

struct ChunkRadius {
    double x0 = 0.0, y0 = 0.0, z0 = 0.0, r2 = 0.0;
    double xp = 0.0, yp = 0.0, zp = 0.0, s2 = 0.0;  // previous point, longest step squared
    bool step_nan = false;
    __device__ __forceinline__ void add(int k, int P, double x, double y, double z,
                                        double *__restrict__ rho, int64_t ld)
    {
        if (k > 0) {
            const double dx = x - x0, dy = y - y0, dz = z - z0;
            const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
            r2 = d2 > r2 ? d2 : r2;
            const double ex = x - xp, ey = y - yp, ez = z - zp;
            const double e2 = fma(ex, ex, fma(ey, ey, ez * ez));
            step_nan = step_nan || !(e2 == e2);
            s2 = e2 > s2 ? e2 : s2;
        }
        xp = x;
        yp = y;
        zp = z;
        if (k % kRadiusChunk == 0) {
            if (k > 0)
                rho[(int64_t)(k / kRadiusChunk - 1) * ld] = sqrt(r2);
            x0 = x;
            y0 = y;
            z0 = z;
            r2 = 0.0;
        }
        if (k == P - 1) {
            rho[(int64_t)(k / kRadiusChunk) * ld] = sqrt(r2);
            rho[(int64_t)radius_chunks(P) * ld] = step_nan ? INFINITY : sqrt(s2);
        }
    }
};

// Eq. 1 for one wire: d = min(lambda, min_j |D - r_j|).
__device__ __forceinline__ double capped_residual(double D, const double *__restrict__ drift,
                                                  int j0, int j1, double lambda)
{
    double d = lambda;
    for (int j = j0; j < j1; ++j) {
        const double e = fabs(D - drift[j]);
        if (e < d)
            d = e;
    }
    return d;
}

}  // namespace cdev

#endif  // COMET_DEVICE_MATH_H
