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
// squared DCA is min(qk, chord(k-1 -> k), chord(k -> k+1)). Point j of seed s is
// track[(c P + j) S + s].
__device__ __forceinline__ double refine_dca2(const double *__restrict__ track, int64_t S, int P,
                                              int64_t s, const double f[8], int k, double qk)
{
    const int64_t PS = (int64_t)P * S;
    const double *t = track + s;
    double cxi, ceta;
    project(f, t[(int64_t)k * S], t[PS + (int64_t)k * S], t[2 * PS + (int64_t)k * S], cxi, ceta);
    double d2 = qk;
    if (k > 0) {
        const int64_t o = (int64_t)(k - 1) * S;
        double xi, eta;
        project(f, t[o], t[PS + o], t[2 * PS + o], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(xi, eta, q, cxi, ceta, qk);
        if (v < d2)
            d2 = v;
    }
    if (k < P - 1) {
        const int64_t o = (int64_t)(k + 1) * S;
        double xi, eta;
        project(f, t[o], t[PS + o], t[2 * PS + o], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2(cxi, ceta, qk, xi, eta, q);
        if (v < d2)
            d2 = v;
    }
    return d2;
}

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
