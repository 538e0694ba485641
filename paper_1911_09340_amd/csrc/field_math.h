// field_math.h -- the magnetic field as a map on a regular grid and the RK4 step that
// reads it (Sec. 2.2.1: tracks are extrapolated through the solenoid's field map).
// Device code shared by the kernels that record tracks in a map.
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 2.2.1.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "device_math.h"

namespace cdev {

// ------------------------------------------------------------------ field map
// B on a regular grid, b[((k ny + j) nx + i) 3 + c] at node (x0 + i dx, y0 + j dy,
// z0 + k dz). A coordinate u = (x - x0) / dx is clamped to [0, n - 1] (NaN to 0),
// i = min(floor(u), n - 2), t = u - i; B is interpolated trilinearly with
// lerp(a, b, t) = fma(t, b - a, a): along x on the four edges (j, k) = (0,0), (1,0),
// (0,1), (1,1), then along y, then along z.
struct FieldMap {
    const double *b;
    int nx, ny, nz;
    double x0, y0, z0, dx, dy, dz;
    int stepper;  // 0: classical RK4 in (x, p); 1: Runge-Kutta-Nystrom in (x, t)
};

__device__ __forceinline__ double lerp(double a, double b, double t) { return fma(t, b - a, a); }

__device__ __forceinline__ void field_cell(double u, int n, int &i, double &t)
{
    if (!(u > 0.0))
        u = 0.0;
    if (u > (double)(n - 1))
        u = (double)(n - 1);
    int k = (int)floor(u);
    if (k > n - 2)
        k = n - 2;
    i = k;
    t = u - (double)k;
}

__device__ __forceinline__ void field_at(const FieldMap &m, double x, double y, double z,
                                         double (&B)[3])
{
    int i, j, k;
    double tu, tv, tw;
    field_cell((x - m.x0) / m.dx, m.nx, i, tu);
    field_cell((y - m.y0) / m.dy, m.ny, j, tv);
    field_cell((z - m.z0) / m.dz, m.nz, k, tw);
    const int64_t sx = 3, sy = 3 * (int64_t)m.nx, sz = 3 * (int64_t)m.nx * m.ny;
    const double *n000 = m.b + k * sz + j * sy + i * sx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double c00 = lerp(n000[c], n000[sx + c], tu);
        const double c10 = lerp(n000[sy + c], n000[sy + sx + c], tu);
        const double c01 = lerp(n000[sz + c], n000[sz + sx + c], tu);
        const double c11 = lerp(n000[sz + sy + c], n000[sz + sy + sx + c], tu);
        B[c] = lerp(lerp(c00, c10, tv), lerp(c01, c11, tv), tw);
    }
}

// The 8 nodes of the last cell a thread read, kept in registers by the recording
// kernels: consecutive stages mostly fall in the same cell (a step moves 2 mm, a cell
// is 25 mm) and a step's first stage sits within ~h^2 |a| of the previous step's last
// one, so reusing the nodes skips dependent global loads. B is computed from the same
// values with the same operations as field_at: the result does not depend on the cache.
struct CellCache {
    double v[24];  // [component][node (0,0,0), (1,0,0), (0,1,0), (1,1,0), (0,0,1), ...]
    int i = -1, j = -1, k = -1;
};

__device__ __forceinline__ void field_at_cached(const FieldMap &m, double x, double y, double z,
                                                double (&B)[3], CellCache &cc)
{
    int i, j, k;
    double tu, tv, tw;
    field_cell((x - m.x0) / m.dx, m.nx, i, tu);
    field_cell((y - m.y0) / m.dy, m.ny, j, tv);
    field_cell((z - m.z0) / m.dz, m.nz, k, tw);
    if (i != cc.i || j != cc.j || k != cc.k) {
        const int64_t sx = 3, sy = 3 * (int64_t)m.nx, sz = 3 * (int64_t)m.nx * m.ny;
        const double *n000 = m.b + k * sz + j * sy + i * sx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cc.v[8 * c + 0] = n000[c];
            cc.v[8 * c + 1] = n000[sx + c];
            cc.v[8 * c + 2] = n000[sy + c];
            cc.v[8 * c + 3] = n000[sy + sx + c];
            cc.v[8 * c + 4] = n000[sz + c];
            cc.v[8 * c + 5] = n000[sz + sx + c];
            cc.v[8 * c + 6] = n000[sz + sy + c];
            cc.v[8 * c + 7] = n000[sz + sy + sx + c];
        }
        cc.i = i;
        cc.j = j;
        cc.k = k;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double c00 = lerp(cc.v[8 * c + 0], cc.v[8 * c + 1], tu);
        const double c10 = lerp(cc.v[8 * c + 2], cc.v[8 * c + 3], tu);
        const double c01 = lerp(cc.v[8 * c + 4], cc.v[8 * c + 5], tu);
        const double c11 = lerp(cc.v[8 * c + 6], cc.v[8 * c + 7], tu);
        B[c] = lerp(lerp(c00, c10, tv), lerp(c01, c11, tv), tw);
    }
}

// RK4 in the map: dx/ds = p inv, dp/ds = g (p x B(x)), inv = 1 / |p of the seed|,
// g = (kappa q) inv; every stage reads B at its own position (x, x + h/2 v1,
// x + h/2 v2, x + h v3); cross product (p_y B_z - p_z B_y, p_z B_x - p_x B_z,
// p_x B_y - p_y B_x); y <- y + h/6 (((k1 + 2 k2) + 2 k3) + k4).
// look(x, y, z, B) reads B: field_at, or field_at_cached in the recording kernels.
template <class Look>
__device__ __forceinline__ void field_force(Look &look, double g, const double (&x)[3],
                                            const double (&p)[3], double (&f)[3])
{
    double B[3];
    look(x[0], x[1], x[2], B);
    f[0] = g * (p[1] * B[2] - p[2] * B[1]);
    f[1] = g * (p[2] * B[0] - p[0] * B[2]);
    f[2] = g * (p[0] * B[1] - p[1] * B[0]);
}

template <class Look>
__device__ __forceinline__ void rk4_field_step_l(Look &look, double inv, double g, double h,
                                                 double (&x)[3], double (&p)[3])
{
    const double hh = 0.5 * h, h6 = h / 6.0;
    double v1[3], f1[3], v2[3], f2[3], v3[3], f3[3], v4[3], f4[3], xs[3], ps[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        v1[c] = p[c] * inv;
    field_force(look, g, x, p, f1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + hh * v1[c];
        ps[c] = p[c] + hh * f1[c];
        v2[c] = ps[c] * inv;
    }
    field_force(look, g, xs, ps, f2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + hh * v2[c];
        ps[c] = p[c] + hh * f2[c];
        v3[c] = ps[c] * inv;
    }
    field_force(look, g, xs, ps, f3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + h * v3[c];
        ps[c] = p[c] + h * f3[c];
        v4[c] = ps[c] * inv;
    }
    field_force(look, g, xs, ps, f4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = x[c] + h6 * (((v1[c] + 2.0 * v2[c]) + 2.0 * v3[c]) + v4[c]);
        p[c] = p[c] + h6 * (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]);
    }
}

__device__ __forceinline__ void rk4_field_step(const FieldMap &m, double inv, double g, double h,
                                               double (&x)[3], double (&p)[3])
{
    auto look = [&](double px, double py, double pz, double (&B)[3]) {
        field_at(m, px, py, pz, B);
    };
    rk4_field_step_l(look, inv, g, h, x, p);
}

// ------------------------------------------------------------------ derivatives
// B at a point and its derivative along a direction (ddx, ddy, ddz): dB = sum over the
// axes of dB/dt_a (dt_a/dx_a) ddx_a, with dt/dx = 1 / spacing, or 0 where the coordinate
// is clamped to the grid (u <= 0, NaN, or u > n - 1: the value is constant there). B is
// computed with the operations of field_at. The derivatives of the trilinear form:
// dB/dt_u = lerp over (v, w) of the x-edge differences, dB/dt_v = lerp over w of the
// y differences, dB/dt_w = the z difference.
__device__ __forceinline__ double cell_slope(double u, int n, double step)
{
    return (!(u > 0.0) || u > (double)(n - 1)) ? 0.0 : 1.0 / step;
}

__device__ __forceinline__ void field_at_dir(const FieldMap &m, const double (&x)[3],
                                             const double (&dx)[3], double (&B)[3],
                                             double (&dB)[3])
{
    const double u = (x[0] - m.x0) / m.dx, v = (x[1] - m.y0) / m.dy, w = (x[2] - m.z0) / m.dz;
    const double du = cell_slope(u, m.nx, m.dx) * dx[0];
    const double dv = cell_slope(v, m.ny, m.dy) * dx[1];
    const double dw = cell_slope(w, m.nz, m.dz) * dx[2];
    int i, j, k;
    double tu, tv, tw;
    field_cell(u, m.nx, i, tu);
    field_cell(v, m.ny, j, tv);
    field_cell(w, m.nz, k, tw);
    const int64_t sx = 3, sy = 3 * (int64_t)m.nx, sz = 3 * (int64_t)m.nx * m.ny;
    const double *n000 = m.b + k * sz + j * sy + i * sx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a000 = n000[c], a100 = n000[sx + c];
        const double a010 = n000[sy + c], a110 = n000[sy + sx + c];
        const double a001 = n000[sz + c], a101 = n000[sz + sx + c];
        const double a011 = n000[sz + sy + c], a111 = n000[sz + sy + sx + c];
        const double c00 = lerp(a000, a100, tu);
        const double c10 = lerp(a010, a110, tu);
        const double c01 = lerp(a001, a101, tu);
        const double c11 = lerp(a011, a111, tu);
        const double e0 = lerp(c00, c10, tv), e1 = lerp(c01, c11, tv);
        B[c] = lerp(e0, e1, tw);
        const double bu = lerp(lerp(a100 - a000, a110 - a010, tv),
                               lerp(a101 - a001, a111 - a011, tv), tw);
        const double bv = lerp(c10 - c00, c11 - c01, tw);
        const double bw = e1 - e0;
        dB[c] = (bu * du + bv * dv) + bw * dw;
    }
}

// f = g (p x B(x)) and its derivative along (dx, dp) with dg the derivative of g:
// df = dg (p x B) + g (dp x B + p x dB).
__device__ __forceinline__ void field_force_dir(const FieldMap &m, double g, double dg,
                                                const double (&x)[3], const double (&p)[3],
                                                const double (&dx)[3], const double (&dp)[3],
                                                double (&f)[3], double (&df)[3])
{
    double B[3], dB[3];
    field_at_dir(m, x, dx, B, dB);
    f[0] = g * (p[1] * B[2] - p[2] * B[1]);
    f[1] = g * (p[2] * B[0] - p[0] * B[2]);
    f[2] = g * (p[0] * B[1] - p[1] * B[0]);
    const double q0 = (dp[1] * B[2] - dp[2] * B[1]) + (p[1] * dB[2] - p[2] * dB[1]);
    const double q1 = (dp[2] * B[0] - dp[0] * B[2]) + (p[2] * dB[0] - p[0] * dB[2]);
    const double q2 = (dp[0] * B[1] - dp[1] * B[0]) + (p[0] * dB[1] - p[1] * dB[0]);
    df[0] = dg * (p[1] * B[2] - p[2] * B[1]) + g * q0;
    df[1] = dg * (p[2] * B[0] - p[0] * B[2]) + g * q1;
    df[2] = dg * (p[0] * B[1] - p[1] * B[0]) + g * q2;
}

// One RK4 step in the map (the primal exactly as rk4_field_step) with its tangent
// (dx, dp) along one seed direction; dinv and dg are that direction's derivatives of
// inv = 1 / |p of the seed| and g = (kappa q) inv.
__device__ __forceinline__ void rk4_field_step_dir(const FieldMap &m, double inv, double g,
                                                   double dinv, double dg, double h,
                                                   double (&x)[3], double (&p)[3],
                                                   double (&dx)[3], double (&dp)[3])
{
    const double hh = 0.5 * h, h6 = h / 6.0;
    double v1[3], f1[3], v2[3], f2[3], v3[3], f3[3], v4[3], f4[3], xs[3], ps[3];
    double dv1[3], df1[3], dv2[3], df2[3], dv3[3], df3[3], dv4[3], df4[3], dxs[3], dps[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v1[c] = p[c] * inv;
        dv1[c] = dp[c] * inv + p[c] * dinv;
    }
    field_force_dir(m, g, dg, x, p, dx, dp, f1, df1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + hh * v1[c];
        ps[c] = p[c] + hh * f1[c];
        v2[c] = ps[c] * inv;
        dxs[c] = dx[c] + hh * dv1[c];
        dps[c] = dp[c] + hh * df1[c];
        dv2[c] = dps[c] * inv + ps[c] * dinv;
    }
    field_force_dir(m, g, dg, xs, ps, dxs, dps, f2, df2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + hh * v2[c];
        ps[c] = p[c] + hh * f2[c];
        v3[c] = ps[c] * inv;
        dxs[c] = dx[c] + hh * dv2[c];
        dps[c] = dp[c] + hh * df2[c];
        dv3[c] = dps[c] * inv + ps[c] * dinv;
    }
    field_force_dir(m, g, dg, xs, ps, dxs, dps, f3, df3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = x[c] + h * v3[c];
        ps[c] = p[c] + h * f3[c];
        v4[c] = ps[c] * inv;
        dxs[c] = dx[c] + h * dv3[c];
        dps[c] = dp[c] + h * df3[c];
        dv4[c] = dps[c] * inv + ps[c] * dinv;
    }
    field_force_dir(m, g, dg, xs, ps, dxs, dps, f4, df4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = x[c] + h6 * (((v1[c] + 2.0 * v2[c]) + 2.0 * v3[c]) + v4[c]);
        p[c] = p[c] + h6 * (((f1[c] + 2.0 * f2[c]) + 2.0 * f3[c]) + f4[c]);
        dx[c] = dx[c] + h6 * (((dv1[c] + 2.0 * dv2[c]) + 2.0 * dv3[c]) + dv4[c]);
        dp[c] = dp[c] + h6 * (((df1[c] + 2.0 * df2[c]) + 2.0 * df3[c]) + df4[c]);
    }
}

// ------------------------------------------------------------------ Runge-Kutta-Nystrom
// Nystrom's fourth-order method for x'' = a(x, x') in arc length, with the unit
// direction t = x' (t = p inv at the seed) and a(x, t) = g (t x B(x)):
//   a1 = a(x, t)
//   xm = (x + hh t) + q8 a1;  a2 = a(xm, t + hh a1);  a3 = a(xm, t + hh a2)
//   xe = (x + h t) + q2 a3;   a4 = a(xe, t + h a3)
//   x <- (x + h t) + q6 ((a1 + a2) + a3);  t <- t + h6 (((a1 + 2 a2) + 2 a3) + a4)
// with hh = 0.5 h, h6 = h / 6, q8 = (h h) / 8, q2 = (h h) * 0.5, q6 = (h h) / 6; a2 and a3
// share one read of B at xm, so a step reads the map three times (RK4: four).
struct RknConsts {
    double h, hh, h6, q8, q2, q6;
};

__device__ __forceinline__ RknConsts rkn_consts(double h)
{
    return RknConsts{h, 0.5 * h, h / 6.0, (h * h) / 8.0, (h * h) * 0.5, (h * h) / 6.0};
}

__device__ __forceinline__ void rkn_accel(double g, const double (&t)[3], const double (&B)[3],
                                          double (&a)[3])
{
    a[0] = g * (t[1] * B[2] - t[2] * B[1]);
    a[1] = g * (t[2] * B[0] - t[0] * B[2]);
    a[2] = g * (t[0] * B[1] - t[1] * B[0]);
}

template <class Look>
__device__ __forceinline__ void rkn_field_step_l(Look &look, const RknConsts &k, double g,
                                                 double (&x)[3], double (&t)[3])
{
    double B[3], a1[3], a2[3], a3[3], a4[3], xs[3], ts[3];
    look(x[0], x[1], x[2], B);
    rkn_accel(g, t, B, a1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = (x[c] + k.hh * t[c]) + k.q8 * a1[c];
        ts[c] = t[c] + k.hh * a1[c];
    }
    look(xs[0], xs[1], xs[2], B);
    rkn_accel(g, ts, B, a2);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        ts[c] = t[c] + k.hh * a2[c];
    rkn_accel(g, ts, B, a3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = (x[c] + k.h * t[c]) + k.q2 * a3[c];
        ts[c] = t[c] + k.h * a3[c];
    }
    look(xs[0], xs[1], xs[2], B);
    rkn_accel(g, ts, B, a4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = (x[c] + k.h * t[c]) + k.q6 * ((a1[c] + a2[c]) + a3[c]);
        t[c] = t[c] + k.h6 * (((a1[c] + 2.0 * a2[c]) + 2.0 * a3[c]) + a4[c]);
    }
}

__device__ __forceinline__ void rkn_field_step(const FieldMap &m, const RknConsts &k, double g,
                                               double (&x)[3], double (&t)[3])
{
    auto look = [&](double px, double py, double pz, double (&B)[3]) {
        field_at(m, px, py, pz, B);
    };
    rkn_field_step_l(look, k, g, x, t);
}

// a = g (t x B) and its derivative along (dt, dB) with dg: dg (t x B) + g (dt x B + t x dB).
__device__ __forceinline__ void rkn_accel_dir(double g, double dg, const double (&t)[3],
                                              const double (&dt)[3], const double (&B)[3],
                                              const double (&dB)[3], double (&a)[3],
                                              double (&da)[3])
{
    rkn_accel(g, t, B, a);
    const double q0 = (dt[1] * B[2] - dt[2] * B[1]) + (t[1] * dB[2] - t[2] * dB[1]);
    const double q1 = (dt[2] * B[0] - dt[0] * B[2]) + (t[2] * dB[0] - t[0] * dB[2]);
    const double q2 = (dt[0] * B[1] - dt[1] * B[0]) + (t[0] * dB[1] - t[1] * dB[0]);
    da[0] = dg * (t[1] * B[2] - t[2] * B[1]) + g * q0;
    da[1] = dg * (t[2] * B[0] - t[0] * B[2]) + g * q1;
    da[2] = dg * (t[0] * B[1] - t[1] * B[0]) + g * q2;
}

// One RKN step (the primal exactly as rkn_field_step) with its tangent (dx, dt) along one
// seed direction; dg is that direction's derivative of g.
__device__ __forceinline__ void rkn_field_step_dir(const FieldMap &m, const RknConsts &k,
                                                   double g, double dg, double (&x)[3],
                                                   double (&t)[3], double (&dx)[3],
                                                   double (&dt)[3])
{
    double B[3], dB[3], a1[3], a2[3], a3[3], a4[3], xs[3], ts[3];
    double da1[3], da2[3], da3[3], da4[3], dxs[3], dts[3];
    field_at_dir(m, x, dx, B, dB);
    rkn_accel_dir(g, dg, t, dt, B, dB, a1, da1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = (x[c] + k.hh * t[c]) + k.q8 * a1[c];
        ts[c] = t[c] + k.hh * a1[c];
        dxs[c] = (dx[c] + k.hh * dt[c]) + k.q8 * da1[c];
        dts[c] = dt[c] + k.hh * da1[c];
    }
    field_at_dir(m, xs, dxs, B, dB);
    rkn_accel_dir(g, dg, ts, dts, B, dB, a2, da2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ts[c] = t[c] + k.hh * a2[c];
        dts[c] = dt[c] + k.hh * da2[c];
    }
    rkn_accel_dir(g, dg, ts, dts, B, dB, a3, da3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xs[c] = (x[c] + k.h * t[c]) + k.q2 * a3[c];
        ts[c] = t[c] + k.h * a3[c];
        dxs[c] = (dx[c] + k.h * dt[c]) + k.q2 * da3[c];
        dts[c] = dt[c] + k.h * da3[c];
    }
    field_at_dir(m, xs, dxs, B, dB);
    rkn_accel_dir(g, dg, ts, dts, B, dB, a4, da4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = (x[c] + k.h * t[c]) + k.q6 * ((a1[c] + a2[c]) + a3[c]);
        t[c] = t[c] + k.h6 * (((a1[c] + 2.0 * a2[c]) + 2.0 * a3[c]) + a4[c]);
        dx[c] = (dx[c] + k.h * dt[c]) + k.q6 * ((da1[c] + da2[c]) + da3[c]);
        dt[c] = dt[c] + k.h6 * (((da1[c] + 2.0 * da2[c]) + 2.0 * da3[c]) + da4[c]);
    }
}

}  // namespace cdev
