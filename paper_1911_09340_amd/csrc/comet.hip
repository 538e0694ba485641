// comet.hip -- seed-scan hot path for MI355X (gfx950): seed grid, RK4 track
// recording, closest-approach distances with the Eq. 1 RSS, seed selection,
// hit classification and the finer re-scan of the grid.
//
// Paper: Yeo, Lee and Kuno, "GPU-accelerated event reconstruction for the COMET
// Phase-I experiment" (arXiv:1911.09340), Sec. 2 (Alg. 1-3, Eq. 1).
//
// Arithmetic follows a fixed evaluation order: the file is compiled with
// -ffp-contract=off, fma() appears only where written, and division and square
// root are the correctly rounded binary64 operations. The same formulas, in the
// same order, define every value the library returns; they are spelled out at
// each device function below.
//
// Data layout in HBM (all device memory owned by the caller):
//   seeds     double[6][S]           SoA, seed fastest
//   track     double[3][P][S]        coordinate, then point, then seed (P = K + 1);
//                                    one wave stores 64 consecutive doubles per row
//   workspace frames double[Wpad][8] (in-plane frame of every wire, padded)
//             dsq    double[n_w][S]  squared capped residual of every (wire, seed)
// No kernel uses atomics on global memory, so every result is deterministic.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "comet.h"

namespace {

constexpr double kKappa = 0.299792458;  // MeV/c per (T mm)
constexpr int kVersion = 100;            // 0.1.0

thread_local char g_last_error[512] = "";

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return status;
}

// Only gfx950 is supported; the answer is cached per device.
int check_device()
{
    static std::mutex mu;
    static int cached[64];  // 0 unknown, 1 ok, -1 unsupported
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(COMET_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64)
        return fail(COMET_EUNSUPPORTED, "device index %d out of range", dev);
    {
        std::lock_guard<std::mutex> lock(mu);
        if (cached[dev] == 0) {
            hipDeviceProp_t prop;
            e = hipGetDeviceProperties(&prop, dev);
            if (e != hipSuccess)
                return fail(COMET_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
            cached[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
            if (cached[dev] < 0)
                snprintf(g_last_error, sizeof(g_last_error), "device %d is %s, not gfx950", dev,
                         prop.gcnArchName);
        }
        if (cached[dev] < 0)
            return COMET_EUNSUPPORTED;
    }
    return COMET_OK;
}

int launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(COMET_EHIP, "%s launch: %s", what, hipGetErrorString(e));
    return COMET_OK;
}

// ------------------------------------------------------------------ profiling
// Optional per-kernel device time: pairs of HIP events recorded around launches.
struct ProfRecord {
    hipEvent_t start, stop;
    int kind;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_records;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Brackets one launch on `stream` with events when profiling is on.
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t stream) : stream_(stream), kind_(kind)
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        if (!g_prof_on)
            return;
        start_ = prof_event();
        stop_ = prof_event();
        if (start_ && stop_)
            hipEventRecord(start_, stream_);
    }
    ~ProfScope()
    {
        if (!start_ || !stop_)
            return;
        hipEventRecord(stop_, stream_);
        std::lock_guard<std::mutex> lock(g_prof_mu);
        g_prof_records.push_back({start_, stop_, kind_});
    }

  private:
    hipStream_t stream_;
    int kind_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

enum { kProfTrack = 0, kProfDca = 1, kProfSum = 2, kProfSelect = 3 };

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int check_config(const comet_config *cfg)
{
    if (!cfg)
        return fail(COMET_EINVAL, "cfg is NULL");
    if (!isfinite(cfg->bz_tesla) || !isfinite(cfg->charge_e))
        return fail(COMET_EINVAL, "bz_tesla and charge_e must be finite");
    if (!finite_pos(cfg->step_mm))
        return fail(COMET_EINVAL, "step_mm must be finite and > 0");
    if (cfg->n_steps < 1 || cfg->n_steps > (1 << 24))
        return fail(COMET_EINVAL, "n_steps must be in [1, 2^24]");
    if (!finite_pos(cfg->lambda_mm))
        return fail(COMET_EINVAL, "lambda_mm must be finite and > 0");
    if (cfg->reserved != 0)
        return fail(COMET_EINVAL, "reserved must be 0");
    return COMET_OK;
}

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

// One thread per seed (Sec. 3.1: the seed set is the product of the component grids).
__global__ void seed_grid_kernel(const double *__restrict__ grid, int n0, int n1, int n2, int n3,
                                 int64_t S, double *__restrict__ seeds)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    const int i3 = (int)(s % n3);
    int64_t rest = s / n3;
    const int i2 = (int)(rest % n2);
    rest /= n2;
    const int i1 = (int)(rest % n1);
    const int i0 = (int)(rest / n1);
    const double v0 = axis_value(grid[6], grid[10], n0, i0);
    const double v1 = axis_value(grid[7], grid[11], n1, i1);
    const double v2 = axis_value(grid[8], grid[12], n2, i2);
    const double v3 = axis_value(grid[9], grid[13], n3, i3);

    const double x0 = grid[0], y0 = grid[1], z0 = grid[2];
    const double px0 = grid[3], py0 = grid[4], pz0 = grid[5];
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
    seeds[0 * S + s] = x0 * ca - y0 * sa;
    seeds[1 * S + s] = y0 * ca + x0 * sa;
    seeds[2 * S + s] = z0;
    seeds[3 * S + s] = v1 * (st * cp);
    seeds[4 * S + s] = v1 * (st * sp);
    seeds[5 * S + s] = v1 * ct;
}

// Finer re-scan around the chosen seed (Sec. 2.1). One thread.
__global__ void refine_grid_kernel(double *__restrict__ grid, int n0, int n1, int n2, int n3,
                                   const int64_t *__restrict__ best)
{
    const int64_t b = best[0];
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
            const double v = axis_value(grid[6 + a], grid[10 + a], n[a], idx[a]);
            grid[6 + a] = v;
            grid[10 + a] = (2.0 * grid[10 + a]) / (double)(n[a] - 1);
        }
    }
}

// ------------------------------------------------------------------ RK4 recording
// Alg. 1, one seed per lane. ODE in path length: dx/ds = p / p0,
// dp/ds = c (p_y, -p_x, 0), c = ((kappa q) B_z) / p0 (as c = ((kappa q) B_z) * inv).
// Classical RK4 with fixed h; y <- y + h/6 (((k1 + 2 k2) + 2 k3) + k4); p_z constant.
// The store of point k writes 64 consecutive doubles per coordinate row per wave.
__global__ __launch_bounds__(256) void rk4_record_kernel(const double *__restrict__ seeds,
                                                         int64_t S, double bz, double charge,
                                                         double h, int K,
                                                         double *__restrict__ track)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double x = seeds[0 * S + s], y = seeds[1 * S + s], z = seeds[2 * S + s];
    double px = seeds[3 * S + s], py = seeds[4 * S + s];
    const double pz = seeds[5 * S + s];
    const double p0 = sqrt((px * px + py * py) + pz * pz);
    const double inv = 1.0 / p0;
    const double c = ((kKappa * charge) * bz) * inv;
    const double hh = 0.5 * h;
    const double h6 = h / 6.0;
    const double vz = pz * inv;
    const int64_t P = (int64_t)K + 1;
    double *tx = track + s;
    double *ty = track + P * S + s;
    double *tz = track + 2 * P * S + s;
    for (int k = 0; k < K; ++k) {
        tx[(int64_t)k * S] = x;
        ty[(int64_t)k * S] = y;
        tz[(int64_t)k * S] = z;
        const double v1x = px * inv, v1y = py * inv;
        const double f1x = c * py, f1y = -(c * px);
        double qx = px + hh * f1x, qy = py + hh * f1y;
        const double v2x = qx * inv, v2y = qy * inv;
        const double f2x = c * qy, f2y = -(c * qx);
        qx = px + hh * f2x;
        qy = py + hh * f2y;
        const double v3x = qx * inv, v3y = qy * inv;
        const double f3x = c * qy, f3y = -(c * qx);
        qx = px + h * f3x;
        qy = py + h * f3y;
        const double v4x = qx * inv, v4y = qy * inv;
        const double f4x = c * qy, f4y = -(c * qx);
        x = x + h6 * (((v1x + 2.0 * v2x) + 2.0 * v3x) + v4x);
        y = y + h6 * (((v1y + 2.0 * v2y) + 2.0 * v3y) + v4y);
        z = z + h6 * (((vz + 2.0 * vz) + 2.0 * vz) + vz);
        px = px + h6 * (((f1x + 2.0 * f2x) + 2.0 * f3x) + f4x);
        py = py + h6 * (((f1y + 2.0 * f2y) + 2.0 * f3y) + f4y);
    }
    tx[(int64_t)K * S] = x;
    ty[(int64_t)K * S] = y;
    tz[(int64_t)K * S] = z;
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

// frames[w] for w < n_w; zero frames pad the array to n_pad entries.
__global__ void frame_kernel(const double *__restrict__ ends, int n_w, int n_pad,
                             double *__restrict__ frames)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_pad)
        return;
    double f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (w < n_w)
        wire_frame(ends + 6 * (int64_t)w, f);
    for (int j = 0; j < 8; ++j)
        frames[8 * (int64_t)w + j] = f[j];
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

// ------------------------------------------------------------------ DCA / Eq. 1
// Work item: a tile of 64 seeds (one per lane) x a group of W * NWV wires. Each of
// the NWV waves owns W wires whose frames sit in scalar registers. The tile's
// track streams through LDS in chunks of C points (loaded once, read by all
// waves), and every lane keeps, per wire, the smallest q seen so far (Alg. 2: the
// recorded state closest to the wire). The first index reaching it is tracked
// either per point (CHUNK_ARGMIN = false: compare + select per point), or per
// chunk (CHUNK_ARGMIN = true: only a running min per point; the chunk holding the
// first minimum is recorded and rescanned from HBM once at the end, recomputing q
// with the same arithmetic so that equality identifies the first index). After
// the last chunk the closest point is refined over its two chords, Eq. 1's capped
// residual is formed, and d^2 is stored to dsq[wire][seed].
//
// Block -> work mapping: consecutive blocks are dealt round-robin over the 8 XCDs;
// the mapping below makes the wire groups of one seed tile consecutive within one
// XCD so that they read the tile's track through the same L2.
template <int W, int NWV, int C, bool CHUNK_ARGMIN>
__global__ __launch_bounds__(64 * NWV) void dca_kernel(
    const double *__restrict__ track, int64_t S, int P, const double *__restrict__ frames,
    int n_w, const int32_t *__restrict__ offsets, const double *__restrict__ drift,
    double lambda, double *__restrict__ dsq, int n_groups, int n_blocks)
{
    __shared__ __align__(16) double lds[3 * C * 64];

    const int b = blockIdx.x;
    const int q8 = n_blocks >> 3, r8 = n_blocks & 7;
    const int xcd = b & 7;
    const int L = xcd * q8 + min(xcd, r8) + (b >> 3);
    const int tile = L / n_groups;
    const int group = L - tile * n_groups;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t s0 = (int64_t)tile * 64;
    const int64_t s = s0 + lane;
    const int wbase = group * (W * NWV) + wave * W;
    const bool active = wbase < n_w;  // wave-uniform

    double f[W][8];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            f[w][j] = frames[8 * (int64_t)(wbase + w) + j];
    double best[W], cmin[W];
    int kbest[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        best[w] = INFINITY;
        cmin[w] = INFINITY;
        kbest[w] = 0;
    }

    // Track chunk staging. Each thread owns UNITS / T slots of two consecutive seeds
    // (16 bytes); the next chunk's loads are issued before the current chunk is
    // scanned, so their latency hides behind the scan.
    constexpr int T = 64 * NWV;
    constexpr int UNITS = 3 * C * 32;
    constexpr int PER_T = (UNITS + T - 1) / T;
    // 16-byte loads when every row start is 16-byte aligned (even S, aligned base)
    const bool pairs = (S & 1) == 0 && ((uintptr_t)track & 15) == 0;
    double2 pre[PER_T];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PER_T; ++u) {
            const int idx = threadIdx.x + u * T;
            const int c = idx / (C * 32);
            const int r = idx - c * (C * 32);
            const int kk = r >> 5;
            const int l2 = (r & 31) * 2;
            const int k = k0 + kk;
            const int64_t ss = s0 + l2;
            double2 v = make_double2(0.0, 0.0);
            if (idx < UNITS && k < P) {
                const double *src = track + ((int64_t)c * P + k) * S + ss;
                if (pairs && ss + 1 < S) {
                    v = *reinterpret_cast<const double2 *>(src);
                } else {
                    if (ss < S)
                        v.x = src[0];
                    if (ss + 1 < S)
                        v.y = src[1];
                }
            }
            pre[u] = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < PER_T; ++u) {
            const int idx = threadIdx.x + u * T;
            if (idx < UNITS)
                *reinterpret_cast<double2 *>(&lds[2 * idx]) = pre[u];
        }
    };

    fetch(0);
    for (int k0 = 0; k0 < P; k0 += C) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + C < P)
            fetch(k0 + C);
        if (active) {
            auto body = [&](int kk) {
                const double x = lds[(0 * C + kk) * 64 + lane];
                const double y = lds[(1 * C + kk) * 64 + lane];
                const double z = lds[(2 * C + kk) * 64 + lane];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    double xi, eta;
                    project(f[w], x, y, z, xi, eta);
                    const double q = fma(xi, xi, eta * eta);
                    if (CHUNK_ARGMIN) {
                        cmin[w] = fmin(cmin[w], q);
                    } else {
                        kbest[w] = q < best[w] ? k0 + kk : kbest[w];
                        best[w] = fmin(best[w], q);
                    }
                }
            };
            const int kn = min(C, P - k0);
            if (kn == C) {
#pragma unroll 4
                for (int kk = 0; kk < C; ++kk)
                    body(kk);
            } else {
                for (int kk = 0; kk < kn; ++kk)
                    body(kk);
            }
            if (CHUNK_ARGMIN) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    if (cmin[w] < best[w]) {
                        best[w] = cmin[w];
                        kbest[w] = k0;
                    }
                    cmin[w] = INFINITY;
                }
            }
        }
    }

    if (!active || s >= S)
        return;
    const int64_t PS = (int64_t)P * S;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int wi = wbase + w;
        if (wi < n_w) {
            int k = kbest[w];
            if (CHUNK_ARGMIN) {
                // first index in the recorded chunk whose q equals the minimum
                const int kend = min(k + C, P);
                int kf = k;
                for (int j = k; j < kend; ++j) {
                    const int64_t o = (int64_t)j * S + s;
                    double xi, eta;
                    project(f[w], track[o], track[PS + o], track[2 * PS + o], xi, eta);
                    if (fma(xi, xi, eta * eta) == best[w]) {
                        kf = j;
                        break;
                    }
                }
                k = kf;
            }
            const double d2 = refine_dca2(track, S, P, s, f[w], k, best[w]);
            const double D = sqrt(d2);
            const double d = capped_residual(D, drift, offsets[wi], offsets[wi + 1], lambda);
            dsq[(int64_t)wi * S + s] = d * d;
        }
    }
}

// Eq. 1's sum over wires in wire order: rss = ((0 + d_0^2) + d_1^2) + ...
__global__ void rss_sum_kernel(const double *__restrict__ dsq, int n_w, int64_t S,
                               double *__restrict__ rss)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double acc = 0.0;
    for (int w = 0; w < n_w; ++w)
        acc = acc + dsq[(int64_t)w * S + s];
    rss[s] = acc;
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

__global__ __launch_bounds__(kSelectThreads) void argmin_kernel(const double *__restrict__ rss,
                                                                int64_t S,
                                                                int64_t *__restrict__ best)
{
    __shared__ double sv[kSelectThreads / 64];
    __shared__ int64_t si[kSelectThreads / 64];
    MinLoc m{INFINITY, -1};
    for (int64_t s = threadIdx.x; s < S; s += kSelectThreads) {
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
    if (wave == 0) {
        MinLoc a{INFINITY, -1};
        if (lane < kSelectThreads / 64) {
            a.v = sv[lane];
            a.i = si[lane];
        }
        for (int off = 32; off > 0; off >>= 1) {
            MinLoc o{__shfl_xor(a.v, off), __shfl_xor(a.i, off)};
            if (beats(o, a))
                a = o;
        }
        if (lane == 0)
            best[0] = a.i;
    }
}

// Classification of the chosen seed (Sec. 2.1): per wire (one thread each), the
// closest recorded point (the chosen track streams through LDS), its chord
// refinement, D, and the hit with the smallest |D - r_j| (first on ties); bit 0 when
// that residual is < lambda, bit 1 when it is within 1e-9 mm of lambda.
constexpr int kClassifyThreads = 1024;
constexpr int kClassifyChunk = 1024;

__global__ __launch_bounds__(kClassifyThreads) void classify_kernel(
    const double *__restrict__ track, int64_t S, int P, const double *__restrict__ ends, int n_w,
    const int32_t *__restrict__ offsets, const double *__restrict__ drift, double lambda,
    const int64_t *__restrict__ best, uint8_t *__restrict__ mask, int32_t *__restrict__ n_border,
    double *__restrict__ dca_out)
{
    __shared__ double pts[3 * kClassifyChunk];
    __shared__ int32_t border;
    if (threadIdx.x == 0)
        border = 0;
    const int64_t b = best[0];
    for (int pass = 0; pass * kClassifyThreads < n_w; ++pass) {
        const int wi = pass * kClassifyThreads + threadIdx.x;
        const bool have = wi < n_w && b >= 0;
        double f[8];
        if (have)
            wire_frame(ends + 6 * (int64_t)wi, f);
        double qb = INFINITY;
        int kb = 0;
        for (int k0 = 0; k0 < P; k0 += kClassifyChunk) {
            const int kn = min(kClassifyChunk, P - k0);
            __syncthreads();
            if (b >= 0)
                for (int i = threadIdx.x; i < 3 * kn; i += kClassifyThreads) {
                    const int c = i / kn, kk = i - c * kn;
                    pts[c * kClassifyChunk + kk] = track[((int64_t)c * P + k0 + kk) * S + b];
                }
            __syncthreads();
            if (have)
                for (int kk = 0; kk < kn; ++kk) {
                    double xi, eta;
                    project(f, pts[kk], pts[kClassifyChunk + kk], pts[2 * kClassifyChunk + kk], xi,
                            eta);
                    const double q = fma(xi, xi, eta * eta);
                    if (q < qb) {
                        qb = q;
                        kb = k0 + kk;
                    }
                }
        }
        if (wi < n_w) {
            const int j0 = offsets[wi], j1 = offsets[wi + 1];
            if (!have) {
                if (mask)
                    for (int j = j0; j < j1; ++j)
                        mask[j] = 0;
                if (dca_out)
                    dca_out[wi] = NAN;
                continue;
            }
            const double D = sqrt(refine_dca2(track, S, P, b, f, kb, qb));
            if (dca_out)
                dca_out[wi] = D;
            int jb = -1;
            double eb = INFINITY;
            for (int j = j0; j < j1; ++j) {
                if (mask)
                    mask[j] = 0;
                const double e = fabs(D - drift[j]);
                if (e < eb) {
                    eb = e;
                    jb = j;
                }
            }
            if (jb >= 0) {
                uint8_t m = 0;
                if (eb < lambda)
                    m |= 1;
                if (fabs(eb - lambda) < 1e-9) {
                    m |= 2;
                    atomicAdd(&border, 1);  // LDS counter: integer, order-independent
                }
                if (mask)
                    mask[jb] = m;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && n_border)
        n_border[0] = border;
}

__global__ void fill_kernel(double *__restrict__ out, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = v;
}

// ------------------------------------------------------------------ DCA variants
struct DcaVariant {
    int w, nwv, c, chunk_argmin;
    void (*kernel)(const double *, int64_t, int, const double *, int, const int32_t *,
                   const double *, double, double *, int, int);
};

const DcaVariant kDcaVariants[] = {
    {4, 8, 32, 1, dca_kernel<4, 8, 32, true>},
    {4, 8, 32, 0, dca_kernel<4, 8, 32, false>},
    {4, 4, 32, 1, dca_kernel<4, 4, 32, true>},
    {2, 8, 32, 1, dca_kernel<2, 8, 32, true>},
    {4, 8, 16, 1, dca_kernel<4, 8, 16, true>},
    {4, 16, 16, 1, dca_kernel<4, 16, 16, true>},
    {5, 8, 32, 1, dca_kernel<5, 8, 32, true>},
    {4, 8, 64, 1, dca_kernel<4, 8, 64, true>},
    {5, 8, 16, 1, dca_kernel<5, 8, 16, true>},
    {6, 8, 16, 1, dca_kernel<6, 8, 16, true>},
    {3, 8, 32, 1, dca_kernel<3, 8, 32, true>},
};
constexpr int kNumDcaVariants = sizeof(kDcaVariants) / sizeof(kDcaVariants[0]);
int g_dca_variant = 0;

constexpr int kMaxWiresPerGroup = 64;  // largest W * NWV in the table above

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Frames are padded so that any variant's last wire group stays in bounds:
// n_groups * (W * NWV) <= n_w + (W * NWV) - 1 <= wire_pad(n_w).
int wire_pad(int n_w)
{
    return ((n_w + 63) / 64) * 64 + kMaxWiresPerGroup;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int comet_version(void) { return kVersion; }

const char *comet_last_error(void) { return g_last_error; }

const char *comet_status_string(int status)
{
    switch (status) {
    case COMET_OK:
        return "ok";
    case COMET_EINVAL:
        return "invalid argument";
    case COMET_EWORKSPACE:
        return "workspace missing or too small";
    case COMET_EHIP:
        return "HIP runtime error";
    case COMET_EUNSUPPORTED:
        return "unsupported device or option";
    default:
        return "unknown status";
    }
}

int comet_seed_grid(const double *grid, const int32_t n[4], double *seeds6, int64_t n_seeds,
                    void *stream)
{
    g_last_error[0] = 0;
    if (!grid || !n || !seeds6)
        return fail(COMET_EINVAL, "comet_seed_grid: NULL pointer");
    int64_t S = 1;
    for (int a = 0; a < 4; ++a) {
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_seed_grid: n[%d] = %d < 1", a, n[a]);
        S *= n[a];
        if (S > ((int64_t)1 << 40))
            return fail(COMET_EINVAL, "comet_seed_grid: grid too large");
    }
    if (S != n_seeds)
        return fail(COMET_EINVAL, "comet_seed_grid: n_seeds %lld != product of n (%lld)",
                    (long long)n_seeds, (long long)S);
    int st = check_device();
    if (st)
        return st;
    const int threads = 256;
    hipLaunchKernelGGL(seed_grid_kernel, dim3((unsigned)((S + threads - 1) / threads)),
                       dim3(threads), 0, (hipStream_t)stream, grid, n[0], n[1], n[2], n[3], S,
                       seeds6);
    return launched("seed_grid_kernel");
}

int comet_refine_grid(double *grid, const int32_t n[4], const int64_t *best, void *stream)
{
    g_last_error[0] = 0;
    if (!grid || !n || !best)
        return fail(COMET_EINVAL, "comet_refine_grid: NULL pointer");
    for (int a = 0; a < 4; ++a)
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_refine_grid: n[%d] = %d < 1", a, n[a]);
    int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(refine_grid_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, grid, n[0],
                       n[1], n[2], n[3], best);
    return launched("refine_grid_kernel");
}

int comet_extrapolate_seeds(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                            double *track_xyz, void *stream)
{
    g_last_error[0] = 0;
    if (!seeds6 || !track_xyz)
        return fail(COMET_EINVAL, "comet_extrapolate_seeds: NULL pointer");
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "comet_extrapolate_seeds: n_seeds = %lld",
                    (long long)n_seeds);
    int st = check_config(cfg);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    const int threads = 256;
    ProfScope prof(kProfTrack, (hipStream_t)stream);
    hipLaunchKernelGGL(rk4_record_kernel, dim3((unsigned)((n_seeds + threads - 1) / threads)),
                       dim3(threads), 0, (hipStream_t)stream, seeds6, n_seeds, cfg->bz_tesla,
                       cfg->charge_e, cfg->step_mm, cfg->n_steps, track_xyz);
    return launched("rk4_record_kernel");
}

size_t comet_dca_workspace_bytes(int64_t n_seeds, int32_t n_wires)
{
    if (n_seeds < 1 || n_wires < 0)
        return 0;
    return align256(sizeof(double) * 8 * (size_t)wire_pad(n_wires)) +
           align256(sizeof(double) * (size_t)n_wires * (size_t)n_seeds);
}

int comet_dca_rss(const double *track_xyz, int64_t n_seeds, int32_t n_points,
                  const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                  const double *drift, int32_t n_hits, const comet_config *cfg, double *rss,
                  void *workspace, size_t workspace_bytes, void *stream)
{
    g_last_error[0] = 0;
    if (!track_xyz || !rss)
        return fail(COMET_EINVAL, "comet_dca_rss: NULL pointer");
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "comet_dca_rss: n_seeds = %lld", (long long)n_seeds);
    if (n_wires < 0 || n_hits < 0)
        return fail(COMET_EINVAL, "comet_dca_rss: negative n_wires or n_hits");
    if (n_wires > 0 && (!wire_ends || !wire_offsets || (n_hits > 0 && !drift)))
        return fail(COMET_EINVAL, "comet_dca_rss: NULL wire or hit array");
    int st = check_config(cfg);
    if (st)
        return st;
    if (n_points != cfg->n_steps + 1)
        return fail(COMET_EINVAL, "comet_dca_rss: n_points %d != n_steps + 1", n_points);
    if ((int64_t)(n_seeds + 63) / 64 * (int64_t)((n_wires + 63) / 64) > (int64_t)1 << 30)
        return fail(COMET_EINVAL, "comet_dca_rss: problem too large for one launch");
    if (n_wires > 0) {
        const size_t need = comet_dca_workspace_bytes(n_seeds, n_wires);
        if (!workspace || workspace_bytes < need)
            return fail(COMET_EWORKSPACE, "comet_dca_rss: workspace %zu < %zu bytes",
                        workspace_bytes, need);
        if (((uintptr_t)workspace & 255) != 0)
            return fail(COMET_EINVAL, "comet_dca_rss: workspace not 256-byte aligned");
    }
    st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    if (n_wires == 0) {
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                           rss, n_seeds, 0.0);
        return launched("fill_kernel");
    }
    const int pad = wire_pad(n_wires);
    double *frames = (double *)workspace;
    double *dsq = (double *)((char *)workspace + align256(sizeof(double) * 8 * (size_t)pad));

    hipLaunchKernelGGL(frame_kernel, dim3((pad + 63) / 64), dim3(64), 0, hs, wire_ends, n_wires,
                       pad, frames);
    st = launched("frame_kernel");
    if (st)
        return st;

    const DcaVariant &v = kDcaVariants[g_dca_variant];
    const int per_group = v.w * v.nwv;
    const int n_groups = (n_wires + per_group - 1) / per_group;
    const int64_t n_tiles = (n_seeds + 63) / 64;
    const int64_t n_blocks = n_tiles * n_groups;
    {
        ProfScope prof(kProfDca, hs);
        hipLaunchKernelGGL(v.kernel, dim3((unsigned)n_blocks), dim3(64 * v.nwv), 0, hs,
                           track_xyz, n_seeds, n_points, (const double *)frames, n_wires,
                           wire_offsets, drift, cfg->lambda_mm, dsq, n_groups, (int)n_blocks);
        st = launched("dca_kernel");
    }
    if (st)
        return st;
    ProfScope prof(kProfSum, hs);
    hipLaunchKernelGGL(rss_sum_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                       (const double *)dsq, n_wires, n_seeds, rss);
    return launched("rss_sum_kernel");
}

int comet_select_classify(const double *rss, int64_t n_seeds, const double *track_xyz,
                          int32_t n_points, const double *wire_ends, int32_t n_wires,
                          const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                          const comet_config *cfg, int32_t top_k, int64_t *best,
                          uint8_t *hit_mask, int32_t *n_borderline, double *dca_best,
                          void *stream)
{
    g_last_error[0] = 0;
    if (!rss || !best)
        return fail(COMET_EINVAL, "comet_select_classify: NULL rss or best");
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "comet_select_classify: n_seeds = %lld", (long long)n_seeds);
    if (top_k != 1)
        return fail(COMET_EUNSUPPORTED, "comet_select_classify: top_k must be 1");
    const bool classify = hit_mask || n_borderline || dca_best;
    if (classify) {
        if (!track_xyz)
            return fail(COMET_EINVAL, "comet_select_classify: NULL track");
        if (n_wires < 0 || n_hits < 0)
            return fail(COMET_EINVAL, "comet_select_classify: negative n_wires or n_hits");
        if (n_wires > 0 && (!wire_ends || !wire_offsets || (n_hits > 0 && !drift)))
            return fail(COMET_EINVAL, "comet_select_classify: NULL wire or hit array");
        int st = check_config(cfg);
        if (st)
            return st;
        if (n_points != cfg->n_steps + 1)
            return fail(COMET_EINVAL, "comet_select_classify: n_points %d != n_steps + 1",
                        n_points);
    }
    int st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    ProfScope prof(kProfSelect, hs);
    hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(kSelectThreads), 0, hs, rss, n_seeds, best);
    st = launched("argmin_kernel");
    if (st || !classify)
        return st;
    hipLaunchKernelGGL(classify_kernel, dim3(1), dim3(kClassifyThreads), 0, hs, track_xyz,
                       n_seeds, n_points, wire_ends, n_wires, wire_offsets, drift, cfg->lambda_mm,
                       (const int64_t *)best, hit_mask, n_borderline, dca_best);
    return launched("classify_kernel");
}

// Tuning hooks (not part of the stable ABI): choose the DCA kernel shape.
int comet_dca_variant_count(void) { return kNumDcaVariants; }

int comet_dca_variant_info(int id, int32_t *w, int32_t *nwv, int32_t *chunk,
                           int32_t *chunk_argmin)
{
    if (id < 0 || id >= kNumDcaVariants || !w || !nwv || !chunk || !chunk_argmin)
        return fail(COMET_EINVAL, "comet_dca_variant_info: bad id or NULL pointer");
    *w = kDcaVariants[id].w;
    *nwv = kDcaVariants[id].nwv;
    *chunk = kDcaVariants[id].c;
    *chunk_argmin = kDcaVariants[id].chunk_argmin;
    return COMET_OK;
}

int comet_profile_begin(void)
{
    std::lock_guard<std::mutex> lock(g_prof_mu);
    for (auto &r : g_prof_records) {
        g_prof_pool.push_back(r.start);
        g_prof_pool.push_back(r.stop);
    }
    g_prof_records.clear();
    g_prof_on = true;
    return COMET_OK;
}

int comet_profile_end(double ms[COMET_PROFILE_KINDS], int64_t launches[COMET_PROFILE_KINDS])
{
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_on = false;
    int status = COMET_OK;
    for (int k = 0; k < COMET_PROFILE_KINDS; ++k) {
        if (ms)
            ms[k] = 0.0;
        if (launches)
            launches[k] = 0;
    }
    for (auto &r : g_prof_records) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) {
            status = fail(COMET_EHIP, "comet_profile_end: %s", hipGetErrorString(e));
        } else if (r.kind >= 0 && r.kind < COMET_PROFILE_KINDS) {
            if (ms)
                ms[r.kind] += t;
            if (launches)
                launches[r.kind] += 1;
        }
        g_prof_pool.push_back(r.start);
        g_prof_pool.push_back(r.stop);
    }
    g_prof_records.clear();
    return status;
}

int comet_dca_set_variant(int id)
{
    if (id < 0 || id >= kNumDcaVariants)
        return fail(COMET_EINVAL, "comet_dca_set_variant: id %d out of range", id);
    g_dca_variant = id;
    return COMET_OK;
}

}  // extern "C"
