// adjoint.hip -- derivatives of the seed scan's RSS with respect to the six seed
// components, and the Levenberg-Marquardt refinement they drive.
//
// Paper: Yeo, Lee and Kuno, "GPU-accelerated event reconstruction for the COMET
// Phase-I experiment" (arXiv:1911.09340). Eq. 1 defines the RSS; Sec. 2.1 notes that
// it is not smooth, which is why the paper scans grids. Piecewise it is smooth: with
// the closest recorded point, the winning chord and each wire's closest hit fixed, D_i
// and the capped residuals are differentiable, and Gauss-Newton steps on the active
// residuals (|D_i - r_j| < lambda) refine a coarse grid's best seed.
//
// Uniform field: one block per seed. Thread 0 records the seed's track into LDS with
// the forward path's cdev::rk4_step, so every D_i, closest index and hit choice equals
// the forward path's. The block then takes the radius of every 16-point window of the
// track, and each wire thread finds its closest point with the forward contract's
// first-index rule, scanning only the windows that a distance bound cannot rule out.
// The derivatives of the recorded points come in closed form: in a uniform B_z the
// RK4 step is linear in the transverse momentum, p_(k+1) = m p_k and
// x_(k+1) = x_k + h inv sigma p_k with complex m and sigma (polynomials in -i h c), so
// x_k = x_0 + h inv sigma G_k p_0 with G_k the geometric sum of m^j, j < k. m^k, G_k and
// dG_k/dm follow by binary powering (O(log k) complex products per active wire), and
// the chain through inv = 1/|p|, c = kappa q B inv and v_z = p_z inv gives the row.
// (The derivatives of the discrete map, as the step-by-step dual numbers of the CPU
// reference give them, up to rounding.)
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

constexpr int kAdjThreads = 256;     // field-map kernel
// uniform-field kernel: four waves per block while its LDS fits in 64 KB, else one
constexpr int kUniThreadsWide = 256;
constexpr int kUniThreadsNarrow = 64;
constexpr int kWindow = 16;  // points per window of the distance bound
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

// The radius of every kWindow-point window of a recorded track in LDS: the largest
// distance of the window's points from its first point (NaN points are passed over;
// they never become a closest point). One thread per window.
__device__ __forceinline__ void window_radii(const double *lx, const double *ly,
                                             const double *lz, int P, double *rho)
{
    const int n_win = (P + kWindow - 1) / kWindow;
    for (int c = threadIdx.x; c < n_win; c += blockDim.x) {
        const int k0 = c * kWindow, k1 = min(P, k0 + kWindow);
        double r2 = 0.0;
        for (int k = k0 + 1; k < k1; ++k) {
            const double dx = lx[k] - lx[k0], dy = ly[k] - ly[k0], dz = lz[k] - lz[k0];
            const double v = fma(dx, dx, fma(dy, dy, dz * dz));
            r2 = v > r2 ? v : r2;
        }
        rho[c] = sqrt(r2);
    }
}

// A wire's DCA to the recorded track (lx, ly, lz; P points) as the forward contract
// takes it: the closest recorded point (first index of the minimum), then the winning
// refinement, the vertex or the interior of an adjacent chord. Returns D; the chord
// starts at point ka with parameter t (0 at the vertex), closest point (pxi, peta) in
// the wire's frame.
//
// The closest point is searched window by window. Every point of window c lies within
// rho[c] of its first point, so its distance to the wire is at least that point's
// minus rho[c]; a window is skipped when this lower bound exceeds the best distance
// known so far (the smallest over every window's first point, then the running
// minimum) by a relative 1e-9 and 1e-9 mm, far above the rounding of q and rho. A
// skipped window holds no point at or below the final minimum, so the first index of
// the minimum is the full scan's; NaN or infinite values never skip.
__device__ __forceinline__ double closest_chord(const double *lx, const double *ly,
                                                const double *lz, const double *rho, int P,
                                                const double (&f)[8], int &ka, double &t,
                                                double &pxi, double &peta)
{
    const int n_win = (P + kWindow - 1) / kWindow;
    // the windows' first points, eight at a time (independent loads and products)
    double ub = INFINITY;
    int c = 0;
    for (; c + 8 <= n_win; c += 8) {
        double qv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = (c + u) * kWindow;
            double xi, eta;
            project(f, lx[k], ly[k], lz[k], xi, eta);
            qv[u] = fma(xi, xi, eta * eta);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            ub = qv[u] < ub ? qv[u] : ub;
    }
    for (; c < n_win; ++c) {
        const int k = c * kWindow;
        double xi, eta;
        project(f, lx[k], ly[k], lz[k], xi, eta);
        const double q = fma(xi, xi, eta * eta);
        ub = q < ub ? q : ub;
    }
    double bound = sqrt(ub);
    int kb = 0;
    double qb = INFINITY;
    for (c = 0; c < n_win; ++c) {
        const int k0 = c * kWindow;
        double xi, eta;
        project(f, lx[k0], ly[k0], lz[k0], xi, eta);
        // skip when sqrt(q0) exceeds rho + bound (compared squared: both sides >= 0)
        const double tb = (rho[c] + bound) * (1.0 + 1e-9) + 1e-9;
        if (fma(xi, xi, eta * eta) > tb * tb)
            continue;
        if (k0 + kWindow <= P) {
            double qv[kWindow];
#pragma unroll
            for (int j = 0; j < kWindow; ++j) {
                project(f, lx[k0 + j], ly[k0 + j], lz[k0 + j], xi, eta);
                qv[j] = fma(xi, xi, eta * eta);
            }
#pragma unroll
            for (int j = 0; j < kWindow; ++j)
                if (qv[j] < qb) {
                    qb = qv[j];
                    kb = k0 + j;
                }
        } else {
            for (int k = k0; k < P; ++k) {
                project(f, lx[k], ly[k], lz[k], xi, eta);
                const double q = fma(xi, xi, eta * eta);
                if (q < qb) {
                    qb = q;
                    kb = k;
                }
            }
        }
        const double sb = sqrt(qb);
        bound = sb < bound ? sb : bound;
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

// Complex numbers for the uniform-field step: a transverse vector (x, y) is x + i y,
// and the magnetic rotation (p_x, p_y) -> c (p_y, -p_x) is multiplication by -i c.
struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx cscale(double s, Cx a) { return {s * a.re, s * a.im}; }

// For n steps of p -> m p: A = m^n, D = dA/dm, G = sum_(j<n) m^j, H = dG/dm.
struct Geo {
    Cx A, D, G, H;
};
// n1 steps then n2 steps (the sums are symmetric in the order).
__device__ __forceinline__ Geo geo_join(const Geo &x, const Geo &y)
{
    return {cmul(x.A, y.A), cadd(cmul(x.D, y.A), cmul(x.A, y.D)), cadd(x.G, cmul(x.A, y.G)),
            cadd(cadd(x.H, cmul(x.D, y.G)), cmul(x.A, y.H))};
}
__device__ __forceinline__ Geo geo_one(Cx m) { return {m, {1.0, 0.0}, {1.0, 0.0}, {0.0, 0.0}}; }
// n >= 0 steps, by binary powering.
__device__ __forceinline__ Geo geo_pow(Cx m, int n)
{
    Geo r{{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    Geo b = geo_one(m);
    while (n > 0) {
        if (n & 1)
            r = geo_join(r, b);
        n >>= 1;
        if (n > 0)
            b = geo_join(b, b);
    }
    return r;
}

// Per-seed constants of the closed-form derivatives: with w = -i h c,
//   m = 1 + w + w^2/2 + w^3/6 + w^4/24   (p_(k+1) = m p_k),
//   sigma = 1 + w/2 + w^2/6 + w^3/24     (x_(k+1) = x_k + h inv sigma p_k),
// and their derivatives with respect to c (dw/dc = -i h).
struct StepPoly {
    Cx m, sigma, dm_dc, dsigma_dc;
};
__device__ __forceinline__ StepPoly step_poly(double h, double c)
{
    const Cx w{0.0, -(h * c)};
    const Cx w2 = cmul(w, w), w3 = cmul(w2, w), w4 = cmul(w3, w);
    const Cx dw{0.0, -h};
    StepPoly sp;
    sp.m = cadd(cadd(cadd(Cx{1.0, 0.0}, w), cadd(cscale(0.5, w2), cscale(1.0 / 6.0, w3))),
                cscale(1.0 / 24.0, w4));
    sp.sigma = cadd(cadd(Cx{1.0, 0.0}, cscale(0.5, w)),
                    cadd(cscale(1.0 / 6.0, w2), cscale(1.0 / 24.0, w3)));
    const Cx dm = cadd(cadd(Cx{1.0, 0.0}, w), cadd(cscale(0.5, w2), cscale(1.0 / 6.0, w3)));
    const Cx ds = cadd(cadd(Cx{0.5, 0.0}, cscale(1.0 / 3.0, w)), cscale(0.125, w2));
    sp.dm_dc = cmul(dm, dw);
    sp.dsigma_dc = cmul(ds, dw);
    return sp;
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
    const double *tracks;   // uniform field: recorded tracks [S][3][K + 1], or NULL
};

// One seed per lane: every seed's track with the forward path's cdev::rk4_step, each
// seed's points contiguous ([S][3][K + 1]) so that an adjoint block loads its seed's
// track whole. The store of point k writes one double of 64 rows per wave; the rows'
// cache lines fill over consecutive points and stay in L2 until they are whole.
__global__ __launch_bounds__(64) void adj_record_kernel(const double *__restrict__ seeds,
                                                        int64_t S, double bz, double charge,
                                                        double h, int K,
                                                        double *__restrict__ tracks)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double x = seeds[0 * S + s], y = seeds[1 * S + s], z = seeds[2 * S + s];
    double px = seeds[3 * S + s], py = seeds[4 * S + s];
    const StepConsts kc = step_consts(px, py, seeds[5 * S + s], bz, charge, h);
    const int P = K + 1;
    double *tx = tracks + (size_t)s * 3 * P, *ty = tx + P, *tz = ty + P;
    for (int j = 0; j < K; ++j) {
        tx[j] = x;
        ty[j] = y;
        tz[j] = z;
        rk4_step(kc, x, y, z, px, py);
    }
    tx[K] = x;
    ty[K] = y;
    tz[K] = z;
}

template <int kUniThreads>
__global__ __launch_bounds__(kUniThreads) void rss_adjoint_kernel(AdjArgs a)
{
    extern __shared__ double lds[];
    const int64_t s = blockIdx.x;
    const int P = a.K + 1;
    double *lx = lds, *ly = lds + P, *lz = lds + 2 * P;
    double *rho = lds + 3 * P;                             // window radii
    double *wbuf = rho + (P + kWindow - 1) / kWindow;      // [kUniThreads][8] per wire

    const int e = a.seed_event ? a.seed_event[s] : 0;
    const int w0 = a.ev_wires ? a.ev_wires[e] : 0;
    const int w1 = a.ev_wires ? a.ev_wires[e + 1] : a.n_w_total;

    const double sx = a.seeds[0 * a.S + s], sy = a.seeds[1 * a.S + s], sz = a.seeds[2 * a.S + s];
    const double spx = a.seeds[3 * a.S + s], spy = a.seeds[4 * a.S + s];
    const double spz = a.seeds[5 * a.S + s];
    const StepConsts kc = step_consts(spx, spy, spz, a.bz, a.charge, a.h);

    if (a.tracks) {  // recorded by adj_record_kernel: load it whole
        const double *src = a.tracks + (size_t)s * 3 * P;
#pragma unroll 4
        for (int i = threadIdx.x; i < 3 * P; i += kUniThreads)
            lds[i] = src[i];
    } else if (threadIdx.x == 0) {
        double x = sx, y = sy, z = sz, px = spx, py = spy;
        for (int j = 0; j < a.K; ++j) {
            lx[j] = x;
            ly[j] = y;
            lz[j] = z;
            rk4_step(kc, x, y, z, px, py);
        }
        lx[a.K] = x;
        ly[a.K] = y;
        lz[a.K] = z;
    }
    __syncthreads();
    window_radii(lx, ly, lz, P, rho);
    __syncthreads();

    // chain from the step's constants to the seed: inv = 1/|p|, c = (kappa q B) inv,
    // v_z = p_z inv; d inv / d p_j = -p_j inv^3
    const StepPoly sp = step_poly(a.h, kc.c);
    const double kqb = (kKappa * a.charge) * a.bz;
    const double inv3 = (kc.inv * kc.inv) * kc.inv;
    const Cx p0c{spx, spy};

    // The sums run in wire order, one quantity per thread (q < 34: rss, grad[6], the
    // packed A[21], b[6]): each round of up to kUniThreads wires leaves every wire's
    // d^2, row and residual in LDS, then the quantity threads add them up. The RSS is
    // thus summed in the forward path's order.
    const int q = threadIdx.x;
    double acc = 0.0;
    int qr = 0, qc = 0;  // row and column of A's entry for 7 <= q < 28
    if (q >= 7 && q < 7 + kTri)
        for (int r = 0, i = 0; r < 6; ++r)
            for (int c2 = r; c2 < 6; ++c2, ++i)
                if (i == q - 7) {
                    qr = r;
                    qc = c2;
                }
    for (int base = w0; base < w1; base += kUniThreads) {
        const int wi = base + threadIdx.x;
        double d2 = 0.0, res_a = 0.0, row[6] = {0, 0, 0, 0, 0, 0};
        if (wi < w1) {
            double f[8];
            wire_frame(a.ends + 6 * (int64_t)wi, f);
            double t, pxi, peta;
            int ka;
            const double D = closest_chord(lx, ly, lz, rho, P, f, ka, t, pxi, peta);
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
            d2 = d * d;
            const int64_t ow = s * (int64_t)a.n_w_total + wi;
            if (a.D)
                a.D[ow] = D;
            if (a.resid)
                a.resid[ow] = res;
            if (active && D > 0.0) {
                res_a = res;
                // dD/dP at the closest point (unit normal from the wire)
                const double nx = (pxi * f[0] + peta * f[4]) / D;
                const double ny = (pxi * f[1] + peta * f[5]) / D;
                const double nz = (pxi * f[2] + peta * f[6]) / D;
                // G and dG/dm at the chord's ends, weighted (1 - t, t)
                const Geo g0 = geo_pow(sp.m, ka);
                const Geo g1 = geo_join(g0, geo_one(sp.m));
                const Cx G = cadd(cscale(1.0 - t, g0.G), cscale(t, g1.G));
                const Cx H = cadd(cscale(1.0 - t, g0.H), cscale(t, g1.H));
                // d(x + i y)/d(p_x0) at fixed c and inv; d/d(p_y0) is i times it
                const Cx sG = cmul(sp.sigma, G);
                const Cx t_p = cscale(a.h * kc.inv, sG);
                // d(x + i y)/dc and d(x + i y)/d inv
                const Cx t_c = cscale(
                    a.h * kc.inv,
                    cmul(cadd(cmul(sp.dsigma_dc, G), cmul(sp.sigma, cmul(H, sp.dm_dc))), p0c));
                const Cx t_inv = cscale(a.h, cmul(sG, p0c));
                const double t_vz = ((double)ka + t) * a.h;  // z_k = z_0 + k h v_z
                const double d_px = t_p.re * nx + t_p.im * ny;
                const double d_py = -t_p.im * nx + t_p.re * ny;
                const double d_c = t_c.re * nx + t_c.im * ny;
                const double d_inv = t_inv.re * nx + t_inv.im * ny;
                const double d_vz = t_vz * nz;
                const double via_inv = (d_inv + kqb * d_c) + spz * d_vz;  // per unit d inv
                row[0] = nx;
                row[1] = ny;
                row[2] = nz;
                row[3] = d_px - via_inv * (spx * inv3);
                row[4] = d_py - via_inv * (spy * inv3);
                row[5] = d_vz * kc.inv - via_inv * (spz * inv3);
            }
            if (a.J)
                for (int r = 0; r < 6; ++r)
                    a.J[ow * 6 + r] = row[r];
        }
        double *wb = wbuf + 8 * threadIdx.x;
        wb[0] = d2;
        wb[7] = res_a;
        for (int r = 0; r < 6; ++r)
            wb[1 + r] = row[r];
        __syncthreads();
        const int n = min(kUniThreads, w1 - base);
        if (q == 0) {
            for (int j = 0; j < n; ++j)
                acc += wbuf[8 * j];
        } else if (q < 7) {
            for (int j = 0; j < n; ++j)
                acc += 2.0 * wbuf[8 * j + 7] * wbuf[8 * j + q];
        } else if (q < 7 + kTri) {
            for (int j = 0; j < n; ++j)
                acc += wbuf[8 * j + 1 + qr] * wbuf[8 * j + 1 + qc];
        } else if (q < 7 + kTri + 6) {
            for (int j = 0; j < n; ++j)
                acc += wbuf[8 * j + 1 + (q - 7 - kTri)] * wbuf[8 * j + 7];
        }
        __syncthreads();
    }
    if (q == 0 && a.rss)
        a.rss[s] = acc;
    else if (q >= 1 && q < 7 && a.grad)
        a.grad[s * 6 + (q - 1)] = acc;
    else if (q >= 7 && q < 7 + kTri && a.A)
        a.A[s * kTri + (q - 7)] = acc;
    else if (q >= 7 + kTri && q < 7 + kTri + 6 && a.b)
        a.b[s * 6 + (q - 7 - kTri)] = acc;
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
    return 3 * P + (P + kWindow - 1) / kWindow > 6 * (kWin + 1) * 3
               ? 3 * P + (P + kWindow - 1) / kWindow
               : 6 * (kWin + 1) * 3;
}

__global__ __launch_bounds__(kAdjThreads) void rss_jacobian_field_kernel(AdjArgs a, FieldMap m)
{
    extern __shared__ double lds[];
    const int64_t s = blockIdx.x;
    const int P = a.K + 1;
    double *lx = lds, *ly = lds + P, *lz = lds + 2 * P;
    double *rho = lds + 3 * P;  // window radii
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
    window_radii(lx, ly, lz, P, rho);
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
        const double D = closest_chord(lx, ly, lz, rho, P, f, ka, t, pxi, peta);
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

size_t adjoint_lds_bytes(int K, int threads)
{
    const int P = K + 1;
    const int n_win = (P + kWindow - 1) / kWindow;
    return sizeof(double) * (3 * (size_t)P + (size_t)n_win + 8 * (size_t)threads);
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
    if (adjoint_lds_bytes(a.K, kUniThreadsWide) <= 65536) {
        hipLaunchKernelGGL(rss_adjoint_kernel<kUniThreadsWide>, dim3((unsigned)a.S),
                           dim3(kUniThreadsWide), adjoint_lds_bytes(a.K, kUniThreadsWide), hs, a);
    } else {
        hipLaunchKernelGGL(rss_adjoint_kernel<kUniThreadsNarrow>, dim3((unsigned)a.S),
                           dim3(kUniThreadsNarrow), adjoint_lds_bytes(a.K, kUniThreadsNarrow), hs,
                           a);
    }
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

size_t comet_lm_workspace_bytes(int64_t n_seeds, int32_t n_steps)
{
    if (n_seeds < 1 || n_steps < 1 || n_steps > kMaxAdjointSteps)
        return 0;
    const size_t S = (size_t)n_seeds;
    return align256(sizeof(double) * 6 * S) + 2 * align256(sizeof(double) * kTri * S) +
           2 * align256(sizeof(double) * 6 * S) + 3 * align256(sizeof(double) * S) +
           2 * align256(sizeof(int32_t) * S) +
           align256(sizeof(double) * 3 * ((size_t)n_steps + 1) * S);
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
    const size_t need = comet_lm_workspace_bytes(n_seeds, cfg->n_steps);
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
    double *tracks = (double *)take(sizeof(double) * 3 * ((size_t)cfg->n_steps + 1) * S);
    if (n_accepted)
        acc = n_accepted;
    // uniform field: every evaluation's tracks are recorded one seed per lane first
    auto record = [&](const double *x) -> int {
        if (fm)
            return COMET_OK;
        hipLaunchKernelGGL(adj_record_kernel, dim3((unsigned)((S + 63) / 64)), dim3(64), 0, hs,
                           x, n_seeds, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, cfg->n_steps,
                           tracks);
        return launched("adj_record_kernel");
    };

    const dim3 grid1((unsigned)((S + 255) / 256)), block1(256);
    AdjArgs a{seeds6, n_seeds, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, cfg->lambda_mm,
              cfg->n_steps, wire_ends, n_wires, wire_offsets, drift, event_wires, seed_event,
              rss, nullptr, A, b, nullptr, nullptr, nullptr, fm ? nullptr : tracks};
    hipLaunchKernelGGL(lm_init_kernel, grid1, block1, 0, hs, n_seeds, mu0, mu, acc);
    st = launched("lm_init_kernel");
    if (!st)
        st = record(seeds6);
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
            st = record(trial);
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
