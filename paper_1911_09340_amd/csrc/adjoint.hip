// adjoint.hip -- derivatives of the seed scan's RSS with respect to the six seed
// components, by a hand-written reverse sweep through the RK4 steps and the active
// DCA chord, and the Levenberg-Marquardt refinement they drive.
//
// Paper: Yeo, Lee and Kuno, "GPU-accelerated event reconstruction for the COMET
// Phase-I experiment" (arXiv:1911.09340). Eq. 1 defines the RSS; Sec. 2.1 notes that
// it is not smooth, which is why the paper scans grids. Piecewise it is smooth: with
// the closest recorded point, the winning chord and each wire's closest hit fixed, D_i
// and the capped residuals are differentiable, and Gauss-Newton steps on the active
// residuals (|D_i - r_j| < lambda) refine a coarse grid's best seed.
//
// One block per seed, one thread per wire. Thread 0 recomputes the seed's track (the
// same cdev::rk4_step as the forward path, so every D_i, closest index and hit choice
// equals the forward path's) into LDS, with the momentum checkpointed every 8 steps.
// Each wire thread finds its closest point and winning chord exactly as the forward
// contract does, then runs the reverse sweep from that chord's far end back to the
// seed, recomputing each 8-step segment's momenta from its checkpoint (RK4 is
// recomputed, never stored per step).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "comet.h"
#include "device_math.h"
#include "field_math.h"
#include "host_common.h"

namespace {

using namespace cdev;
using namespace chost;

constexpr int kAdjThreads = 256;
constexpr int kCheckEvery = 8;
constexpr int kTri = 21;  // packed upper triangle of a symmetric 6x6 matrix

// Index of (r, c), r <= c, in the packed row-major upper triangle.
__host__ __device__ constexpr int tri(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// Chord a -> b as in cdev::chord_distance2, also returning the chord parameter t of
// the closest point (0 or 1 when clamped).
__device__ __forceinline__ double chord_distance2_t(double axi, double aeta, double qa,
                                                    double bxi, double beta, double qb,
                                                    double &t, double &pxi, double &peta)
{
    const double uxi = bxi - axi, ueta = beta - aeta;
    const double g = fma(axi, uxi, aeta * ueta);
    const double den = fma(uxi, uxi, ueta * ueta);
    if (!(g < 0.0)) {
        t = 0.0;
        pxi = axi;
        peta = aeta;
        return qa;
    }
    if (-g >= den) {
        t = 1.0;
        pxi = bxi;
        peta = beta;
        return qb;
    }
    t = -g / den;
    pxi = fma(t, uxi, axi);
    peta = fma(t, ueta, aeta);
    return fma(pxi, pxi, peta * peta);
}

// A wire's DCA to the recorded track (lx, ly, lz; P points) as the forward contract
// takes it: the closest recorded point (first index of the minimum), then the winning
// refinement, the vertex or the interior of an adjacent chord. Returns D; the chord
// starts at point ka with parameter t (0 at the vertex), closest point (pxi, peta) in
// the wire's frame.
__device__ __forceinline__ double closest_chord(const double *lx, const double *ly,
                                                const double *lz, int P, const double (&f)[8],
                                                int &ka, double &t, double &pxi, double &peta)
{
    int kb = 0;
    double qb = INFINITY;
    for (int k = 0; k < P; ++k) {
        double xi, eta;
        project(f, lx[k], ly[k], lz[k], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        if (q < qb) {
            qb = q;
            kb = k;
        }
    }
    double cxi, ceta;
    project(f, lx[kb], ly[kb], lz[kb], cxi, ceta);
    double d2 = qb;
    pxi = cxi;
    peta = ceta;
    t = 0.0;
    ka = kb;
    if (kb > 0) {
        double xi, eta, tt, qx, qe;
        project(f, lx[kb - 1], ly[kb - 1], lz[kb - 1], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2_t(xi, eta, q, cxi, ceta, qb, tt, qx, qe);
        if (v < d2) {
            d2 = v;
            ka = kb - 1;
            t = tt;
            pxi = qx;
            peta = qe;
        }
    }
    if (kb < P - 1) {
        double xi, eta, tt, qx, qe;
        project(f, lx[kb + 1], ly[kb + 1], lz[kb + 1], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        const double v = chord_distance2_t(cxi, ceta, qb, xi, eta, q, tt, qx, qe);
        if (v < d2) {
            d2 = v;
            ka = kb;
            t = tt;
            pxi = qx;
            peta = qe;
        }
    }
    return sqrt(d2);
}

// Reverse sweep of one RK4 step (cdev::rk4_step) at start momentum (px, py): maps the
// adjoint of the step's output momentum (pxb, pyb) and position (xb, yb, zb) to the
// adjoint of its input, accumulating the adjoints of inv, c and vz. Positions enter
// the step linearly with unit Jacobian, so their adjoint passes through unchanged.
__device__ __forceinline__ void rk4_step_adjoint(const StepConsts &k, double px, double py,
                                                 double xb, double yb, double zb, double &pxb,
                                                 double &pyb, double &invb, double &cb,
                                                 double &vzb)
{
    const double c = k.c, inv = k.inv, h = k.h, hh = k.hh, h6 = k.h6;
    // forward stage values
    const double f1x = c * py, f1y = -(c * px);
    const double q2x = px + hh * f1x, q2y = py + hh * f1y;
    const double f2x = c * q2y, f2y = -(c * q2x);
    const double q3x = px + hh * f2x, q3y = py + hh * f2y;
    const double f3x = c * q3y, f3y = -(c * q3x);
    const double q4x = px + h * f3x, q4y = py + h * f3y;
    // output adjoints spread over the stages (weights 1, 2, 2, 1 times h/6)
    const double v1bx = h6 * xb, v1by = h6 * yb;
    const double v2bx = 2.0 * v1bx, v2by = 2.0 * v1by;
    double f1bx = h6 * pxb, f1by = h6 * pyb;
    double f2bx = 2.0 * f1bx, f2by = 2.0 * f1by;
    double f3bx = f2bx, f3by = f2by;
    const double f4bx = f1bx, f4by = f1by;
    vzb += 6.0 * h6 * zb;
    double pnx = pxb, pny = pyb;
    // stage 4: v4 = q4 inv, f4 = c (q4y, -q4x)
    {
        const double qbx = v1bx * inv + c * (-f4by), qby = v1by * inv + c * f4bx;
        invb += v1bx * q4x + v1by * q4y;
        cb += f4bx * q4y - f4by * q4x;
        pnx += qbx;
        pny += qby;
        f3bx += h * qbx;
        f3by += h * qby;
    }
    // stage 3
    {
        const double qbx = v2bx * inv + c * (-f3by), qby = v2by * inv + c * f3bx;
        invb += v2bx * q3x + v2by * q3y;
        cb += f3bx * q3y - f3by * q3x;
        pnx += qbx;
        pny += qby;
        f2bx += hh * qbx;
        f2by += hh * qby;
    }
    // stage 2
    {
        const double qbx = v2bx * inv + c * (-f2by), qby = v2by * inv + c * f2bx;
        invb += v2bx * q2x + v2by * q2y;
        cb += f2bx * q2y - f2by * q2x;
        pnx += qbx;
        pny += qby;
        f1bx += hh * qbx;
        f1by += hh * qby;
    }
    // stage 1: v1 = p inv, f1 = c (py, -px)
    pnx += v1bx * inv + c * (-f1by);
    pny += v1by * inv + c * f1bx;
    invb += v1bx * px + v1by * py;
    cb += f1bx * py - f1by * px;
    pxb = pnx;
    pyb = pny;
}

// Block reduction of NV doubles per thread into thread 0 (fixed order).
template <int NV>
__device__ void block_sum(double (&v)[NV], double *scratch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < NV; ++i)
        for (int off = 32; off > 0; off >>= 1)
            v[i] += __shfl_down(v[i], off);
    __syncthreads();
    if (lane == 0)
        for (int i = 0; i < NV; ++i)
            scratch[wave * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) {
            double s = scratch[i];
            for (int w = 1; w < kAdjThreads / 64; ++w)
                s += scratch[w * NV + i];
            v[i] = s;
        }
}

// Per-seed outputs: rss, grad[6] = sum over active wires of 2 e_i J_i, A = sum J_i J_i^T
// (packed triangle), b = sum J_i e_i. Optional per-wire outputs D, resid (signed
// residual of the closest hit, NaN without hits), J (zero rows for capped wires).
// Seed s uses event seed_event[s] (0 if seed_event is NULL); event e owns wires
// [ev_wires[e], ev_wires[e+1]) (all wires if ev_wires is NULL).
struct AdjArgs {
    const double *seeds;
    int64_t S;
    double bz, charge, h, lambda;
    int K;
    const double *ends;
    int n_w_total;
    const int32_t *offsets;
    const double *drift;
    const int32_t *ev_wires;
    const int32_t *seed_event;
    double *rss, *grad, *A, *b;
    double *D, *resid, *J;  // indexed by global wire: [S][n_w_total]
};

__global__ __launch_bounds__(kAdjThreads) void rss_adjoint_kernel(AdjArgs a)
{
    extern __shared__ double lds[];
    const int64_t s = blockIdx.x;
    const int P = a.K + 1;
    double *lx = lds, *ly = lds + P, *lz = lds + 2 * P;
    double *ck = lds + 3 * P;                        // checkpoints: (px, py) pairs
    const int n_ck = a.K / kCheckEvery + 1;
    double *scratch = ck + 2 * n_ck;                 // reductions

    const int e = a.seed_event ? a.seed_event[s] : 0;
    const int w0 = a.ev_wires ? a.ev_wires[e] : 0;
    const int w1 = a.ev_wires ? a.ev_wires[e + 1] : a.n_w_total;

    const double sx = a.seeds[0 * a.S + s], sy = a.seeds[1 * a.S + s], sz = a.seeds[2 * a.S + s];
    const double spx = a.seeds[3 * a.S + s], spy = a.seeds[4 * a.S + s];
    const double spz = a.seeds[5 * a.S + s];
    const StepConsts kc = step_consts(spx, spy, spz, a.bz, a.charge, a.h);

    if (threadIdx.x == 0) {
        double x = sx, y = sy, z = sz, px = spx, py = spy;
        for (int j = 0; j < a.K; ++j) {
            lx[j] = x;
            ly[j] = y;
            lz[j] = z;
            if (j % kCheckEvery == 0) {
                ck[2 * (j / kCheckEvery)] = px;
                ck[2 * (j / kCheckEvery) + 1] = py;
            }
            rk4_step(kc, x, y, z, px, py);
        }
        lx[a.K] = x;
        ly[a.K] = y;
        lz[a.K] = z;
        if (a.K % kCheckEvery == 0) {
            ck[2 * (a.K / kCheckEvery)] = px;
            ck[2 * (a.K / kCheckEvery) + 1] = py;
        }
    }
    __syncthreads();

    // per-thread partial sums: rss, grad[6], A[21], b[6]
    double acc[1 + 6 + kTri + 6];
    for (int i = 0; i < 1 + 6 + kTri + 6; ++i)
        acc[i] = 0.0;

    for (int wi = w0 + threadIdx.x; wi < w1; wi += kAdjThreads) {
        double f[8];
        wire_frame(a.ends + 6 * (int64_t)wi, f);
        double t, pxi, peta;
        int ka;
        const double D = closest_chord(lx, ly, lz, P, f, ka, t, pxi, peta);
        // closest hit and Eq. 1's capped residual
        double eb = INFINITY, res = NAN;
        for (int j = a.offsets[wi]; j < a.offsets[wi + 1]; ++j) {
            const double r = D - a.drift[j];
            if (fabs(r) < eb) {
                eb = fabs(r);
                res = r;
            }
        }
        const bool active = eb < a.lambda;
        const double d = active ? eb : a.lambda;
        acc[0] += d * d;
        const int64_t ow = s * (int64_t)a.n_w_total + wi;
        if (a.D)
            a.D[ow] = D;
        if (a.resid)
            a.resid[ow] = res;
        double row[6] = {0, 0, 0, 0, 0, 0};
        if (active && D > 0.0) {
            // dD/dP at the closest point, spread over the chord's two ends
            const double nx = (pxi * f[0] + peta * f[4]) / D;
            const double ny = (pxi * f[1] + peta * f[5]) / D;
            const double nz = (pxi * f[2] + peta * f[6]) / D;
            const int kend = t > 0.0 ? ka + 1 : ka;  // farthest point with a cotangent
            double xb = (kend == ka ? 1.0 - t : t) * nx;
            double yb = (kend == ka ? 1.0 - t : t) * ny;
            double zb = (kend == ka ? 1.0 - t : t) * nz;
            double pxb = 0.0, pyb = 0.0, invb = 0.0, cb = 0.0, vzb = 0.0;
            // reverse over segments [g * 8, g * 8 + 8) from the one holding kend - 1
            for (int g = (kend - 1) / kCheckEvery; kend > 0 && g >= 0; --g) {
                const int k0 = g * kCheckEvery;
                double mpx[kCheckEvery], mpy[kCheckEvery];
                {
                    double x = 0.0, y = 0.0, z = 0.0, px = ck[2 * g], py = ck[2 * g + 1];
#pragma unroll
                    for (int j = 0; j < kCheckEvery; ++j) {
                        mpx[j] = px;
                        mpy[j] = py;
                        rk4_step(kc, x, y, z, px, py);
                    }
                }
#pragma unroll
                for (int j = kCheckEvery - 1; j >= 0; --j) {
                    const int k = k0 + j;  // step k maps point k to point k + 1
                    if (k < kend) {
                        rk4_step_adjoint(kc, mpx[j], mpy[j], xb, yb, zb, pxb, pyb, invb, cb,
                                         vzb);
                        if (k == ka && kend != ka) {
                            xb += (1.0 - t) * nx;
                            yb += (1.0 - t) * ny;
                            zb += (1.0 - t) * nz;
                        }
                    }
                }
            }
            // constants: vz = pz inv, c = ((kappa q) B) inv, inv = 1 / |p|
            double gpz = vzb * kc.inv;
            invb += vzb * spz;
            invb += cb * ((kKappa * a.charge) * a.bz);
            const double p0b = -invb * kc.inv * kc.inv;
            const double p0 = 1.0 / kc.inv;
            row[0] = xb;
            row[1] = yb;
            row[2] = zb;
            row[3] = pxb + p0b * spx / p0;
            row[4] = pyb + p0b * spy / p0;
            row[5] = gpz + p0b * spz / p0;
            for (int r = 0; r < 6; ++r) {
                acc[1 + r] += 2.0 * res * row[r];
                acc[1 + 6 + kTri + r] += row[r] * res;
                for (int c2 = r; c2 < 6; ++c2)
                    acc[1 + 6 + tri(r, c2)] += row[r] * row[c2];
            }
        }
        if (a.J)
            for (int r = 0; r < 6; ++r)
                a.J[ow * 6 + r] = row[r];
    }

    block_sum(acc, scratch);
    if (threadIdx.x == 0) {
        if (a.rss)
            a.rss[s] = acc[0];
        if (a.grad)
            for (int r = 0; r < 6; ++r)
                a.grad[s * 6 + r] = acc[1 + r];
        if (a.A)
            for (int r = 0; r < kTri; ++r)
                a.A[s * kTri + r] = acc[1 + 6 + r];
        if (a.b)
            for (int r = 0; r < 6; ++r)
                a.b[s * 6 + r] = acc[1 + 6 + kTri + r];
    }
}

// ------------------------------------------------------------------ field map
// Derivatives in a field map (Sec. 2.2.1), in forward mode: the reverse sweep above
// relies on the uniform field's rotation; in a map each stage's force depends on the
// position through B(x), and six tangents (one per seed component) carried along the
// RK4 steps with dB/dx from the trilinear interpolation give dP_k/d(seed) directly.
//
// One block per seed. Thread 0 records the track into LDS (rk4_field_step, as
// comet_extrapolate_seeds_field); each thread takes up to kFieldWiresPerThread of the
// event's wires, finds each wire's chord (closest_chord), its closest hit and Eq. 1's
// capped residual, and keeps the active ones (ka, t, unit normal, e). Then threads 0-5
// step the six tangents window by window (kWin steps), writing the position tangents
// of the window's points to LDS, and after each window every thread forms the rows
// J_i = n . ((1 - t) dP_ka + t dP_ka+1) of its wires whose chord starts in the window.
constexpr int kWin = 64;
constexpr int kFieldWiresPerThread = 4;
constexpr int kMaxFieldWires = kAdjThreads * kFieldWiresPerThread;

__host__ __device__ constexpr int field_region(int P)
{
    return 3 * P > 6 * (kWin + 1) * 3 ? 3 * P : 6 * (kWin + 1) * 3;
}

__global__ __launch_bounds__(kAdjThreads) void rss_jacobian_field_kernel(AdjArgs a, FieldMap m)
{
    extern __shared__ double lds[];
    const int64_t s = blockIdx.x;
    const int P = a.K + 1;
    double *lx = lds, *ly = lds + P, *lz = lds + 2 * P;
    double *buf = lds;  // after the wires' chords are taken: [6][kWin + 1][3]
    double *scratch = lds + field_region(P);

    const int e = a.seed_event ? a.seed_event[s] : 0;
    const int w0 = a.ev_wires ? a.ev_wires[e] : 0;
    const int w1 = a.ev_wires ? a.ev_wires[e + 1] : a.n_w_total;
    if (w1 - w0 > kMaxFieldWires) {  // block-uniform: more wires than the records hold
        if (threadIdx.x == 0) {
            if (a.rss)
                a.rss[s] = NAN;
            for (int r = 0; r < 6; ++r) {
                if (a.grad)
                    a.grad[s * 6 + r] = NAN;
                if (a.b)
                    a.b[s * 6 + r] = NAN;
            }
            if (a.A)
                for (int r = 0; r < kTri; ++r)
                    a.A[s * kTri + r] = NAN;
        }
        return;
    }
    double sd[6];
    for (int c = 0; c < 6; ++c)
        sd[c] = a.seeds[c * a.S + s];
    const double p0 = sqrt((sd[3] * sd[3] + sd[4] * sd[4]) + sd[5] * sd[5]);
    const double inv = 1.0 / p0;
    const double g = (kKappa * a.charge) * inv;

    const bool rkn = m.stepper == 1;
    const RknConsts kn = rkn_consts(a.h);
    if (threadIdx.x == 0) {
        double x[3] = {sd[0], sd[1], sd[2]}, p[3] = {sd[3], sd[4], sd[5]};
        if (rkn)  // the unit direction
            for (int c = 0; c < 3; ++c)
                p[c] = p[c] * inv;
        for (int j = 0; j < a.K; ++j) {
            lx[j] = x[0];
            ly[j] = x[1];
            lz[j] = x[2];
            if (rkn)
                rkn_field_step(m, kn, g, x, p);
            else
                rk4_field_step(m, inv, g, a.h, x, p);
        }
        lx[a.K] = x[0];
        ly[a.K] = x[1];
        lz[a.K] = x[2];
    }
    __syncthreads();

    double acc[1 + 6 + kTri + 6];
    for (int i = 0; i < 1 + 6 + kTri + 6; ++i)
        acc[i] = 0.0;
    int rk[kFieldWiresPerThread], rw[kFieldWiresPerThread];
    double rt[kFieldWiresPerThread], rn0[kFieldWiresPerThread], rn1[kFieldWiresPerThread];
    double rn2[kFieldWiresPerThread], re[kFieldWiresPerThread];
#pragma unroll
    for (int r = 0; r < kFieldWiresPerThread; ++r) {
        rk[r] = -1;
        rw[r] = 0;
        rt[r] = rn0[r] = rn1[r] = rn2[r] = re[r] = 0.0;
        const int wi = w0 + threadIdx.x + r * kAdjThreads;
        if (wi >= w1)
            continue;
        double f[8];
        wire_frame(a.ends + 6 * (int64_t)wi, f);
        double t, pxi, peta;
        int ka;
        const double D = closest_chord(lx, ly, lz, P, f, ka, t, pxi, peta);
        double eb = INFINITY, res = NAN;
        for (int j = a.offsets[wi]; j < a.offsets[wi + 1]; ++j) {
            const double rr = D - a.drift[j];
            if (fabs(rr) < eb) {
                eb = fabs(rr);
                res = rr;
            }
        }
        const bool active = eb < a.lambda;
        const double d = active ? eb : a.lambda;
        acc[0] += d * d;
        const int64_t ow = s * (int64_t)a.n_w_total + wi;
        if (a.D)
            a.D[ow] = D;
        if (a.resid)
            a.resid[ow] = res;
        if (active && D > 0.0) {
            rk[r] = ka;
            rw[r] = wi;
            rt[r] = t;
            rn0[r] = (pxi * f[0] + peta * f[4]) / D;
            rn1[r] = (pxi * f[1] + peta * f[5]) / D;
            rn2[r] = (pxi * f[2] + peta * f[6]) / D;
            re[r] = res;
        } else if (a.J) {
            for (int c = 0; c < 6; ++c)
                a.J[ow * 6 + c] = 0.0;
        }
    }
    __syncthreads();  // the track's LDS becomes the tangent buffer

    // threads 0-5: seed direction c = threadIdx.x; p0, inv, g differentiated at the seed
    double x[3] = {sd[0], sd[1], sd[2]}, p[3] = {sd[3], sd[4], sd[5]};
    double dx[3] = {0.0, 0.0, 0.0}, dp[3] = {0.0, 0.0, 0.0};
    double dinv = 0.0, dg = 0.0;
    const int dir = threadIdx.x;
    if (dir < 3) {
        dx[dir] = 1.0;
    } else if (dir < 6) {
        dp[dir - 3] = 1.0;
        const double dp0 = sd[dir] / p0;
        dinv = -(dp0 * inv) * inv;
        dg = (kKappa * a.charge) * dinv;
    }
    if (rkn)  // (p, dp) become the unit direction and its tangent
        for (int c = 0; c < 3; ++c) {
            dp[c] = dp[c] * inv + p[c] * dinv;
            p[c] = p[c] * inv;
        }
    const int n_win = a.K / kWin + 1;
    for (int w = 0; w < n_win; ++w) {
        const int base = w * kWin;
        const int last = min(base + kWin, a.K);
        if (dir < 6) {
            double *bc = buf + dir * (kWin + 1) * 3;
            for (int k = base; k <= last; ++k) {
                bc[(k - base) * 3 + 0] = dx[0];
                bc[(k - base) * 3 + 1] = dx[1];
                bc[(k - base) * 3 + 2] = dx[2];
                if (k < last) {
                    if (rkn)
                        rkn_field_step_dir(m, kn, g, dg, x, p, dx, dp);
                    else
                        rk4_field_step_dir(m, inv, g, dinv, dg, a.h, x, p, dx, dp);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kFieldWiresPerThread; ++r) {
            if (rk[r] < 0 || rk[r] / kWin != w)
                continue;
            const int o = rk[r] - base;
            const double t = rt[r];
            double row[6];
            for (int c = 0; c < 6; ++c) {
                const double *bc = buf + c * (kWin + 1) * 3 + o * 3;
                double gx = bc[0], gy = bc[1], gz = bc[2];
                if (t > 0.0) {
                    gx = (1.0 - t) * gx + t * bc[3];
                    gy = (1.0 - t) * gy + t * bc[4];
                    gz = (1.0 - t) * gz + t * bc[5];
                }
                row[c] = (rn0[r] * gx + rn1[r] * gy) + rn2[r] * gz;
            }
            const double res = re[r];
            for (int q = 0; q < 6; ++q) {
                acc[1 + q] += 2.0 * res * row[q];
                acc[1 + 6 + kTri + q] += row[q] * res;
                for (int c2 = q; c2 < 6; ++c2)
                    acc[1 + 6 + tri(q, c2)] += row[q] * row[c2];
            }
            if (a.J) {
                const int64_t ow = s * (int64_t)a.n_w_total + rw[r];
                for (int c = 0; c < 6; ++c)
                    a.J[ow * 6 + c] = row[c];
            }
        }
        __syncthreads();
    }

    block_sum(acc, scratch);
    if (threadIdx.x == 0) {
        if (a.rss)
            a.rss[s] = acc[0];
        if (a.grad)
            for (int r = 0; r < 6; ++r)
                a.grad[s * 6 + r] = acc[1 + r];
        if (a.A)
            for (int r = 0; r < kTri; ++r)
                a.A[s * kTri + r] = acc[1 + 6 + r];
        if (a.b)
            for (int r = 0; r < 6; ++r)
                a.b[s * 6 + r] = acc[1 + 6 + kTri + r];
    }
}

// ------------------------------------------------------------------ Levenberg-Marquardt
// Step proposal: solve (A + mu diag(A)) delta = -b by Cholesky (6x6); trial = seed +
// delta; ok = 0 when the matrix is not positive definite (trial = seed).
__global__ void lm_propose_kernel(int64_t S, const double *__restrict__ seeds,
                                  const double *__restrict__ A, const double *__restrict__ b,
                                  const double *__restrict__ mu, double *__restrict__ trial,
                                  int32_t *__restrict__ ok)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double M[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) {
            const double v = A[s * kTri + tri(r, c)];
            M[r][c] = v;
            M[c][r] = v;
        }
    for (int r = 0; r < 6; ++r)
        M[r][r] = M[r][r] + mu[s] * M[r][r];
    double L[6][6] = {};
    bool pd = true;
    for (int i = 0; i < 6 && pd; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = M[i][j];
            for (int k = 0; k < j; ++k)
                v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 0.0)) {
                    pd = false;
                    break;
                }
                L[i][i] = sqrt(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    double x[6] = {0, 0, 0, 0, 0, 0};
    if (pd) {
        double y[6];
        for (int i = 0; i < 6; ++i) {
            double v = -b[s * 6 + i];
            for (int k = 0; k < i; ++k)
                v -= L[i][k] * y[k];
            y[i] = v / L[i][i];
        }
        for (int i = 5; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 6; ++k)
                v -= L[k][i] * x[k];
            x[i] = v / L[i][i];
        }
    }
    for (int r = 0; r < 6; ++r)
        trial[r * S + s] = seeds[r * S + s] + x[r];
    ok[s] = pd ? 1 : 0;
}

// Accept the trial when it lowers the RSS (mu /= 10), otherwise keep the seed (mu *= 10).
__global__ void lm_accept_kernel(int64_t S, double *__restrict__ seeds,
                                 const double *__restrict__ trial, double *__restrict__ rss,
                                 const double *__restrict__ rss_t, double *__restrict__ A,
                                 const double *__restrict__ A_t, double *__restrict__ b,
                                 const double *__restrict__ b_t, double *__restrict__ mu,
                                 const int32_t *__restrict__ ok, int32_t *__restrict__ n_acc)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    if (ok[s] && rss_t[s] < rss[s]) {
        for (int r = 0; r < 6; ++r) {
            seeds[r * S + s] = trial[r * S + s];
            b[s * 6 + r] = b_t[s * 6 + r];
        }
        for (int r = 0; r < kTri; ++r)
            A[s * kTri + r] = A_t[s * kTri + r];
        rss[s] = rss_t[s];
        mu[s] = mu[s] / 10.0;
        n_acc[s] += 1;
    } else {
        mu[s] = mu[s] * 10.0;
    }
}

__global__ void lm_init_kernel(int64_t S, double mu0, double *__restrict__ mu,
                               int32_t *__restrict__ n_acc)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    mu[s] = mu0;
    n_acc[s] = 0;
}

constexpr int kMaxAdjointSteps = 2400;

size_t adjoint_lds_bytes(int K)
{
    const int P = K + 1;
    const int n_ck = K / kCheckEvery + 1;
    return sizeof(double) * (3 * (size_t)P + 2 * (size_t)n_ck + (kAdjThreads / 64) * 34);
}

int check_adjoint_args(const char *who, const double *seeds6, int64_t n_seeds,
                       const comet_config *cfg, const double *wire_ends, int32_t n_wires,
                       const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                       const int32_t *event_wires, const int32_t *seed_event)
{
    if (!seeds6)
        return fail(COMET_EINVAL, "%s: NULL seeds", who);
    if (n_seeds < 1 || n_seeds > (1 << 30))
        return fail(COMET_EINVAL, "%s: n_seeds = %lld", who, (long long)n_seeds);
    if (n_wires < 0 || n_hits < 0)
        return fail(COMET_EINVAL, "%s: negative n_wires or n_hits", who);
    if (n_wires > 0 && (!wire_ends || !wire_offsets || (n_hits > 0 && !drift)))
        return fail(COMET_EINVAL, "%s: NULL wire or hit array", who);
    if ((event_wires == nullptr) != (seed_event == nullptr))
        return fail(COMET_EINVAL, "%s: event_wires and seed_event go together", who);
    int st = check_config(cfg);
    if (st)
        return st;
    if (cfg->n_steps > kMaxAdjointSteps)
        return fail(COMET_EUNSUPPORTED, "%s: n_steps %d > %d", who, cfg->n_steps,
                    kMaxAdjointSteps);
    return COMET_OK;
}

size_t field_jacobian_lds_bytes(int K)
{
    return sizeof(double) * ((size_t)field_region(K + 1) + (kAdjThreads / 64) * 34);
}

// The uniform-field reverse sweep, or the field map's forward tangents when fm is set.
int launch_adjoint(const AdjArgs &a, hipStream_t hs, const FieldMap *fm = nullptr)
{
    if (fm) {
        hipLaunchKernelGGL(rss_jacobian_field_kernel, dim3((unsigned)a.S), dim3(kAdjThreads),
                           field_jacobian_lds_bytes(a.K), hs, a, *fm);
        return launched("rss_jacobian_field_kernel");
    }
    const size_t lds = adjoint_lds_bytes(a.K);
    hipLaunchKernelGGL(rss_adjoint_kernel, dim3((unsigned)a.S), dim3(kAdjThreads), lds, hs, a);
    return launched("rss_adjoint_kernel");
}

FieldMap field_map_of(const comet_field *f)
{
    return FieldMap{f->b, f->nx, f->ny, f->nz, f->x0, f->y0, f->z0, f->dx, f->dy, f->dz,
                    f->stepper};
}

}  // namespace

extern "C" {

int comet_rss_adjoint(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                      const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                      const double *drift, int32_t n_hits, const int32_t *event_wires,
                      const int32_t *seed_event, double *rss, double *grad, double *jtj,
                      double *jte, double *dca, double *resid, double *jac, void *stream)
{
    clear_error();
    int st = check_adjoint_args("comet_rss_adjoint", seeds6, n_seeds, cfg, wire_ends, n_wires,
                                wire_offsets, drift, n_hits, event_wires, seed_event);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    AdjArgs a{seeds6, n_seeds, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, cfg->lambda_mm,
              cfg->n_steps, wire_ends, n_wires, wire_offsets, drift, event_wires, seed_event,
              rss, grad, jtj, jte, dca, resid, jac};
    return launch_adjoint(a, (hipStream_t)stream);
}

size_t comet_lm_workspace_bytes(int64_t n_seeds)
{
    if (n_seeds < 1)
        return 0;
    const size_t S = (size_t)n_seeds;
    return align256(sizeof(double) * 6 * S) + 2 * align256(sizeof(double) * kTri * S) +
           2 * align256(sizeof(double) * 6 * S) + 3 * align256(sizeof(double) * S) +
           2 * align256(sizeof(int32_t) * S);
}

}  // extern "C"

namespace {

int lm_refine_impl(const char *who, double *seeds6, int64_t n_seeds, const comet_config *cfg,
                   const FieldMap *fm, const double *wire_ends, int32_t n_wires,
                   const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                   const int32_t *event_wires, const int32_t *seed_event, int32_t n_iter,
                   double mu0, double *rss, int32_t *n_accepted, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    int st = check_adjoint_args(who, seeds6, n_seeds, cfg, wire_ends, n_wires, wire_offsets,
                                drift, n_hits, event_wires, seed_event);
    if (st)
        return st;
    if (!rss)
        return fail(COMET_EINVAL, "%s: NULL rss", who);
    if (n_iter < 0 || n_iter > 1000)
        return fail(COMET_EINVAL, "%s: n_iter must be in [0, 1000]", who);
    if (!(mu0 > 0.0) || !isfinite(mu0))
        return fail(COMET_EINVAL, "%s: mu0 must be finite and > 0", who);
    const size_t need = comet_lm_workspace_bytes(n_seeds);
    if (!workspace || workspace_bytes < need)
        return fail(COMET_EWORKSPACE, "%s: workspace %zu < %zu bytes", who, workspace_bytes,
                    need);
    if (((uintptr_t)workspace & 255) != 0)
        return fail(COMET_EINVAL, "%s: workspace not 256-byte aligned", who);
    st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    const size_t S = (size_t)n_seeds;
    char *p = (char *)workspace;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return r;
    };
    double *trial = (double *)take(sizeof(double) * 6 * S);
    double *A = (double *)take(sizeof(double) * kTri * S);
    double *A_t = (double *)take(sizeof(double) * kTri * S);
    double *b = (double *)take(sizeof(double) * 6 * S);
    double *b_t = (double *)take(sizeof(double) * 6 * S);
    double *rss_t = (double *)take(sizeof(double) * S);
    double *mu = (double *)take(sizeof(double) * S);
    double *unused = (double *)take(sizeof(double) * S);
    (void)unused;
    int32_t *ok = (int32_t *)take(sizeof(int32_t) * S);
    int32_t *acc = (int32_t *)take(sizeof(int32_t) * S);
    if (n_accepted)
        acc = n_accepted;

    const dim3 grid1((unsigned)((S + 255) / 256)), block1(256);
    AdjArgs a{seeds6, n_seeds, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, cfg->lambda_mm,
              cfg->n_steps, wire_ends, n_wires, wire_offsets, drift, event_wires, seed_event,
              rss, nullptr, A, b, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL(lm_init_kernel, grid1, block1, 0, hs, n_seeds, mu0, mu, acc);
    st = launched("lm_init_kernel");
    if (!st)
        st = launch_adjoint(a, hs, fm);
    AdjArgs at = a;
    at.seeds = trial;
    at.rss = rss_t;
    at.A = A_t;
    at.b = b_t;
    for (int it = 0; it < n_iter && st == COMET_OK; ++it) {
        hipLaunchKernelGGL(lm_propose_kernel, grid1, block1, 0, hs, n_seeds,
                           (const double *)seeds6, (const double *)A, (const double *)b,
                           (const double *)mu, trial, ok);
        st = launched("lm_propose_kernel");
        if (!st)
            st = launch_adjoint(at, hs, fm);
        if (!st) {
            hipLaunchKernelGGL(lm_accept_kernel, grid1, block1, 0, hs, n_seeds, seeds6,
                               (const double *)trial, rss, (const double *)rss_t, A,
                               (const double *)A_t, b, (const double *)b_t, mu,
                               (const int32_t *)ok, acc);
            st = launched("lm_accept_kernel");
        }
    }
    return st;
}

}  // namespace

extern "C" {

int comet_lm_refine(double *seeds6, int64_t n_seeds, const comet_config *cfg,
                    const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                    const double *drift, int32_t n_hits, const int32_t *event_wires,
                    const int32_t *seed_event, int32_t n_iter, double mu0, double *rss,
                    int32_t *n_accepted, void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    return lm_refine_impl("comet_lm_refine", seeds6, n_seeds, cfg, nullptr, wire_ends, n_wires,
                          wire_offsets, drift, n_hits, event_wires, seed_event, n_iter, mu0,
                          rss, n_accepted, workspace, workspace_bytes, stream);
}

int comet_rss_jacobian_field(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                             const comet_field *field, const double *wire_ends, int32_t n_wires,
                             const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                             const int32_t *event_wires, const int32_t *seed_event, double *rss,
                             double *grad, double *jtj, double *jte, double *dca, double *resid,
                             double *jac, void *stream)
{
    clear_error();
    int st = check_adjoint_args("comet_rss_jacobian_field", seeds6, n_seeds, cfg, wire_ends,
                                n_wires, wire_offsets, drift, n_hits, event_wires, seed_event);
    if (st)
        return st;
    st = check_field("comet_rss_jacobian_field", field);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    AdjArgs a{seeds6, n_seeds, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, cfg->lambda_mm,
              cfg->n_steps, wire_ends, n_wires, wire_offsets, drift, event_wires, seed_event,
              rss, grad, jtj, jte, dca, resid, jac};
    const FieldMap m = field_map_of(field);
    return launch_adjoint(a, (hipStream_t)stream, &m);
}

int comet_lm_refine_field(double *seeds6, int64_t n_seeds, const comet_config *cfg,
                          const comet_field *field, const double *wire_ends, int32_t n_wires,
                          const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                          const int32_t *event_wires, const int32_t *seed_event, int32_t n_iter,
                          double mu0, double *rss, int32_t *n_accepted, void *workspace,
                          size_t workspace_bytes, void *stream)
{
    clear_error();
    const int st = check_field("comet_lm_refine_field", field);
    if (st)
        return st;
    const FieldMap m = field_map_of(field);
    return lm_refine_impl("comet_lm_refine_field", seeds6, n_seeds, cfg, &m, wire_ends,
                          n_wires, wire_offsets, drift, n_hits, event_wires, seed_event, n_iter,
                          mu0, rss, n_accepted, workspace, workspace_bytes, stream);
}

}  // extern "C"
