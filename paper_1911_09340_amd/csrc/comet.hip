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

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "comet.h"
#include "dca_scan.h"
#include "device_math.h"
#include "host_common.h"

namespace {

constexpr int kVersion = 100;  // 0.1.0

using namespace cdev;
using namespace chost;

// ------------------------------------------------------------------ seed grid
// One thread per seed (Sec. 3.1: the seed set is the product of the component grids).
__global__ void seed_grid_kernel(const double *__restrict__ grid, int n0, int n1, int n2, int n3,
                                 int64_t S, double *__restrict__ seeds)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double st[6];
    seed_from_grid(grid, n0, n1, n2, n3, s, st);
    for (int c = 0; c < 6; ++c)
        seeds[c * S + s] = st[c];
}

// Finer re-scan around the chosen seed (Sec. 2.1). One thread.
__global__ void refine_grid_kernel(double *__restrict__ grid, int n0, int n1, int n2, int n3,
                                   const int64_t *__restrict__ best)
{
    refine_grid_desc(grid, n0, n1, n2, n3, best[0]);
}

// ------------------------------------------------------------------ RK4 recording
// Alg. 1, one seed per lane (the step is cdev::rk4_step). The store of point k
// writes 64 consecutive doubles per coordinate row per wave. With rho set, the chunk
// radii of the track (as chunk_radius_kernel computes them, layout [window][S]) are
// taken while recording, so the scan needs no second read of the track.
__global__ __launch_bounds__(256) void rk4_record_kernel(const double *__restrict__ seeds,
                                                         int64_t S, double bz, double charge,
                                                         double h, int K,
                                                         double *__restrict__ track,
                                                         double *__restrict__ rho)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double x = seeds[0 * S + s], y = seeds[1 * S + s], z = seeds[2 * S + s];
    double px = seeds[3 * S + s], py = seeds[4 * S + s];
    const double pz = seeds[5 * S + s];
    const cdev::StepConsts k = cdev::step_consts(px, py, pz, bz, charge, h);
    const int64_t P = (int64_t)K + 1;
    double *tx = track + s;
    double *ty = track + P * S + s;
    double *tz = track + 2 * P * S + s;
    cdev::ChunkRadius cr;
    double *rs = rho ? rho + s : nullptr;
    for (int j = 0; j < K; ++j) {
        tx[(int64_t)j * S] = x;
        ty[(int64_t)j * S] = y;
        tz[(int64_t)j * S] = z;
        if (rs)
            cr.add(j, K + 1, x, y, z, rs, S);
        cdev::rk4_step(k, x, y, z, px, py);
    }
    tx[(int64_t)K * S] = x;
    ty[(int64_t)K * S] = y;
    tz[(int64_t)K * S] = z;
    if (rs)
        cr.add(K, K + 1, x, y, z, rs, S);
}

// Chunk radii of every seed's track (ChunkRadius: window n holds points 16 n ...
// min(16 n + 16, P - 1), rho = the largest distance from its first point): one thread
// per (seed, window), consecutive threads on consecutive seeds, so that every load
// of a block reads one contiguous row segment.
__global__ __launch_bounds__(256) void chunk_radius_kernel(const double *__restrict__ track,
                                                           int64_t S, int P,
                                                           double *__restrict__ rho)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    const int64_t PS = (int64_t)P * S;
    const int nch = cdev::radius_chunks(P);
    double s2 = 0.0;  // the longest step of this thread's windows
    bool step_nan = false;
    for (int n = blockIdx.y; n < nch; n += gridDim.y) {
        const int k0 = n * cdev::kRadiusChunk;
        const int k1 = min(k0 + cdev::kRadiusChunk, P - 1);
        const int64_t o0 = (int64_t)k0 * S + s;
        const double x0 = track[o0], y0 = track[PS + o0], z0 = track[2 * PS + o0];
        double r2 = 0.0;
        double xp = x0, yp = y0, zp = z0;
#pragma unroll 4
        for (int k = k0 + 1; k <= k1; ++k) {
            const int64_t o = (int64_t)k * S + s;
            const double x = track[o], y = track[PS + o], z = track[2 * PS + o];
            const double dx = x - x0, dy = y - y0, dz = z - z0;
            const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
            r2 = d2 > r2 ? d2 : r2;
            const double ex = x - xp, ey = y - yp, ez = z - zp;
            const double e2 = fma(ex, ex, fma(ey, ey, ez * ez));
            step_nan = step_nan || !(e2 == e2);
            s2 = e2 > s2 ? e2 : s2;
            xp = x;
            yp = y;
            zp = z;
        }
        rho[(int64_t)n * S + s] = sqrt(r2);
    }
    // row nch: the longest step over all windows (the row starts at 0; for non-negative
    // doubles the order of the bit patterns is the order of the values)
    const double st = step_nan ? INFINITY : sqrt(s2);
    atomicMax(reinterpret_cast<unsigned long long *>(rho + (int64_t)nch * S + s),
              (unsigned long long)__double_as_longlong(st));
}

// ------------------------------------------------------------------ wire frames
// frames[w] for w < n_w; zero frames pad the array to n_pad entries. key[w]: the
// azimuth of the wire's midpoint (+inf for the padding), the order in which the wide
// DCA form deals wires to waves.
__global__ void frame_kernel(const double *__restrict__ ends, int n_w, int n_pad,
                             double *__restrict__ frames, float *__restrict__ key)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_pad)
        return;
    double f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    float k = INFINITY;
    if (w < n_w) {
        const double *e = ends + 6 * (int64_t)w;
        wire_frame(e, f);
        k = atan2f((float)(e[1] + e[4]), (float)(e[0] + e[3]));
        if (k != k)
            k = 4.0f;  // a NaN endpoint: after every finite azimuth, before the padding
    }
    for (int j = 0; j < 8; ++j)
        frames[8 * (int64_t)w + j] = f[j];
    key[w] = k;
}

// The wide form's wire order: slot r of frames_sorted / wire_of holds the wire of rank r
// in (key, index) order. Wires near each other in azimuth share a wave, so the wave's
// wires need nearly the same track chunks. The order changes which wave evaluates a
// wire, never a result.
// caps[r]: the largest drift distance of the wire in slot r (-1 for a wire without hits
// and for the padding), for the wide form's cap of the distance bound.
__global__ void wire_order_kernel(const double *__restrict__ frames, const float *__restrict__ key,
                                  int n_pad, int n_w, const int32_t *__restrict__ offsets,
                                  const double *__restrict__ drift,
                                  double *__restrict__ frames_sorted,
                                  int32_t *__restrict__ wire_of, double *__restrict__ caps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad)
        return;
    const float ki = key[i];
    int rank = 0;
    for (int j = 0; j < n_pad; ++j) {
        const float kj = key[j];
        rank += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
    }
    for (int j = 0; j < 8; ++j)
        frames_sorted[8 * (int64_t)rank + j] = frames[8 * (int64_t)i + j];
    wire_of[rank] = i;
    double rmax = -1.0;
    if (i < n_w)
        for (int j = offsets[i]; j < offsets[i + 1]; ++j)
            rmax = drift[j] > rmax ? drift[j] : rmax;
    caps[rank] = rmax;
}

// ------------------------------------------------------------------ DCA / Eq. 1
// Work item: a tile of 64 seeds (one per lane) x a group of W * NWV wires, scanned by
// cdev::TileScan (dca_scan.h); d^2 of every (wire, seed) goes to dsq[wire][seed].
//
// Block -> work mapping: consecutive blocks are dealt round-robin over the 8 XCDs;
// with xcd_remap the wire groups of one seed tile become consecutive within one
// XCD so that they can read the tile's track through the same L2 (without it,
// consecutive block indices take consecutive groups).
//
// Registers are capped for 4 waves per SIMD (two 8-wave blocks or one 16-wave block
// per CU); the frames live in scalar registers, so only the running minima, the
// staged point and the prefetch buffer occupy vector registers.
template <int W, int NWV, int C, bool CHUNK_ARGMIN, bool DIRECT, int SUP>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(4))) void dca_kernel(
    const double *__restrict__ track, int64_t S, int P, const double *__restrict__ frames,
    int n_w, const int32_t *__restrict__ offsets, const double *__restrict__ drift,
    double lambda, const double *__restrict__ rho, double *__restrict__ dsq, int n_groups,
    int n_blocks, int xcd_remap, unsigned long long *counter)
{
    using Scan = std::conditional_t<DIRECT, TileScanDirect<W, C, CHUNK_ARGMIN, true, SUP>,
                                    TileScan<W, NWV, C, CHUNK_ARGMIN>>;
    using ScanFar =
        std::conditional_t<DIRECT, TileScanDirect<W, C, CHUNK_ARGMIN, false, SUP>, Scan>;
    __shared__ __align__(16) double lds[Scan::kLdsDoubles];

    const int b = blockIdx.x;
    const int q8 = n_blocks >> 3, r8 = n_blocks & 7;
    const int xcd = b & 7;
    const int L = xcd_remap ? xcd * q8 + min(xcd, r8) + (b >> 3) : b;
    // wave-uniform (the division runs on the vector unit; keep the result scalar)
    const int tile = __builtin_amdgcn_readfirstlane(L / n_groups);
    const int group = L - tile * n_groups;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t s0 = (int64_t)tile * 64;
    const int n_valid = (int)min((int64_t)64, S - s0);
    const int wbase = group * (W * NWV) + wave * W;
    const int nw = max(0, min(W, n_w - wbase));  // wave-uniform

    double f[W][8];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            f[w][j] = frames[8 * (int64_t)(wbase + w) + j];

    const int64_t PS = (int64_t)P * S;
    // 16-byte loads when every row start is 16-byte aligned (even S, aligned base)
    const bool pairs = (S & 1) == 0 && ((uintptr_t)track & 15) == 0;
    double d2[W];
    // 32-bit buffer offsets reach every point of the tile when P S doubles span < 4 GiB
    if (!DIRECT || (int64_t)P * S < ((int64_t)1 << 29) - 64)
        Scan::run(track + s0, track + PS + s0, track + 2 * PS + s0, S, P, n_valid, pairs, f, nw,
                  offsets + (nw > 0 ? wbase : 0), drift, lambda, rho + s0, S, counter, lds, d2);
    else
        ScanFar::run(track + s0, track + PS + s0, track + 2 * PS + s0, S, P, n_valid, pairs, f,
                     nw, offsets + (nw > 0 ? wbase : 0), drift, lambda, rho + s0, S, counter, lds,
                     d2);
    if (lane < n_valid)
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (w < nw)
                dsq[(int64_t)(wbase + w) * S + s0 + lane] = d2[w];
}

// The wide form (TileScanWide): a block is a 64-seed tile x NWV waves of W wires in
// azimuth order; the block's frames are copied to LDS once. WPE: waves per SIMD the
// registers are sized for; EXACT: the first index of the minimum tracked point by point;
// HS (with CAP and EXACT): a needed chunk in HS parts, each tested per wire before it is
// scanned (0: no parts).
template <int W, int NWV, int SUP, int WPE, int NB = 0, bool CAP = false, bool EXACT = false,
          int HS = 0>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(WPE))) void dca_wide_kernel(
    const double *__restrict__ track, int64_t S, int P, const double *__restrict__ frames_sorted,
    const int32_t *__restrict__ wire_of, const double *__restrict__ caps, int n_w,
    const int32_t *__restrict__ offsets, const double *__restrict__ drift, double lambda,
    const double *__restrict__ rho, double *__restrict__ dsq, int n_groups, int n_blocks,
    int xcd_remap, unsigned long long *counter)
{
    __shared__ __align__(16) double fl[NWV * W * 8];
    const int b = blockIdx.x;
    const int q8 = n_blocks >> 3, r8 = n_blocks & 7;
    const int xcd = b & 7;
    const int L = xcd_remap ? xcd * q8 + min(xcd, r8) + (b >> 3) : b;
    const int tile = __builtin_amdgcn_readfirstlane(L / n_groups);
    const int group = L - tile * n_groups;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t s0 = (int64_t)tile * 64;
    const int n_valid = (int)min((int64_t)64, S - s0);
    const int gbase = group * (W * NWV);
    const int wbase = gbase + wave * W;
    const int nw = max(0, min(W, n_w - wbase));  // wave-uniform
    for (int i = threadIdx.x; i < NWV * W * 8; i += 64 * NWV)
        fl[i] = frames_sorted[8 * (int64_t)gbase + i];
    __syncthreads();
    const int64_t PS = (int64_t)P * S;
    double d2[W];
    // NB > 0: the latency-hiding form (batches of NB chunk tests, double-buffered halves)
    using Near = std::conditional_t<(NB > 0), TileScanWideP<W, (NB > 0 ? NB : 1), true, CAP>,
                                    TileScanWide<W, SUP, true, CAP, EXACT, HS>>;
    using Far = std::conditional_t<(NB > 0), TileScanWideP<W, (NB > 0 ? NB : 1), false, CAP>,
                                   TileScanWide<W, SUP, false, CAP, EXACT, HS>>;
    if ((int64_t)P * S < ((int64_t)1 << 29) - 64)
        Near::run(track + s0, track + PS + s0, track + 2 * PS + s0, S, P, n_valid,
                  fl + wave * W * 8, nw, wire_of + wbase, offsets, drift, lambda, rho + s0, S,
                  counter, d2, caps + wbase);
    else
        Far::run(track + s0, track + PS + s0, track + 2 * PS + s0, S, P, n_valid,
                 fl + wave * W * 8, nw, wire_of + wbase, offsets, drift, lambda, rho + s0, S,
                 counter, d2, caps + wbase);
    if (lane < n_valid)
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (w < nw)
                dsq[(int64_t)wire_of[wbase + w] * S + s0 + lane] = d2[w];
}

// Eq. 1's sum over wires in wire order: rss = ((0 + d_0^2) + d_1^2) + ...
__global__ void rss_sum_kernel(const double *__restrict__ dsq, int n_w, int64_t S,
                               double *__restrict__ rss)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    // loads run ahead in batches of 8 (independent addresses); the adds stay in wire order
    const double *p = dsq + s;
    double acc = 0.0;
    int w = 0;
    for (; w + 8 <= n_w; w += 8) {
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            v[i] = p[(int64_t)(w + i) * S];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            acc = acc + v[i];
    }
    for (; w < n_w; ++w)
        acc = acc + p[(int64_t)w * S];
    rss[s] = acc;
}

// ------------------------------------------------------------------ selection
__global__ __launch_bounds__(kSelectThreads) void argmin_kernel(const double *__restrict__ rss,
                                                                int64_t S,
                                                                int64_t *__restrict__ best)
{
    const int64_t b = block_argmin(rss, S);
    if (threadIdx.x == 0)
        best[0] = b;
}

// Classification of the chosen seed (Sec. 2.1): per wire (one thread each), the
// closest recorded point (the chosen track streams through LDS), its chord
// refinement, D, and the hit with the smallest |D - r_j| (first on ties); bit 0 when
// that residual is < lambda, bit 1 when it is within 1e-9 mm of lambda.
constexpr int kClassifyThreads = 1024;
constexpr int kClassifyChunk = 1024;
constexpr int kClassifyLanes = 4;  // threads per wire (within one wave)
constexpr int kClassifyWires = kClassifyThreads / kClassifyLanes;

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
    // kClassifyLanes threads per wire, each taking every kClassifyLanes-th point; their
    // (q, k) minima are combined with the lower index winning ties, which gives the first
    // index of the minimum, as one thread scanning in order would.
    const int lane_of_wire = threadIdx.x % kClassifyLanes;
    for (int pass = 0; pass * kClassifyWires < n_w; ++pass) {
        const int wi = pass * kClassifyWires + threadIdx.x / kClassifyLanes;
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
                for (int kk = lane_of_wire; kk < kn; kk += kClassifyLanes) {
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
#pragma unroll
        for (int off = 1; off < kClassifyLanes; off <<= 1) {
            const double oq = __shfl_xor(qb, off);
            const int ok = __shfl_xor(kb, off);
            if (oq < qb || (oq == qb && ok < kb)) {
                qb = oq;
                kb = ok;
            }
        }
        if (lane_of_wire == 0 && wi < n_w) {
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
    int w, nwv, c, chunk_argmin, xcd_remap, direct, sup;
    void (*kernel)(const double *, int64_t, int, const double *, int, const int32_t *,
                   const double *, double, const double *, double *, int, int, int,
                   unsigned long long *);
    // the wide form (direct == 2): frames in azimuth order and each slot's wire
    void (*wide)(const double *, int64_t, int, const double *, const int32_t *, const double *,
                 int, const int32_t *, const double *, double, const double *, double *, int,
                 int, int, unsigned long long *) = nullptr;
    int wpe = 4;
    const char *name = "";  // the kernel as a profiler names it
};

const DcaVariant kDcaVariants[] = {
    {6, 8, 16, 1, 1, 0, 1, dca_kernel<6, 8, 16, true, false, 1>, nullptr, 4, "dca_kernel<6, 8, 16, true, false, 1>"},
    {6, 8, 16, 1, 0, 0, 1, dca_kernel<6, 8, 16, true, false, 1>, nullptr, 4, "dca_kernel<6, 8, 16, true, false, 1>"},
    {6, 16, 16, 1, 1, 0, 1, dca_kernel<6, 16, 16, true, false, 1>, nullptr, 4, "dca_kernel<6, 16, 16, true, false, 1>"},
    {5, 16, 16, 1, 1, 0, 1, dca_kernel<5, 16, 16, true, false, 1>, nullptr, 4, "dca_kernel<5, 16, 16, true, false, 1>"},
    {4, 16, 16, 1, 1, 0, 1, dca_kernel<4, 16, 16, true, false, 1>, nullptr, 4, "dca_kernel<4, 16, 16, true, false, 1>"},
    {4, 8, 32, 0, 1, 0, 1, dca_kernel<4, 8, 32, false, false, 1>, nullptr, 4, "dca_kernel<4, 8, 32, false, false, 1>"},
    {4, 8, 32, 1, 1, 0, 1, dca_kernel<4, 8, 32, true, false, 1>, nullptr, 4, "dca_kernel<4, 8, 32, true, false, 1>"},
    {4, 8, 16, 1, 1, 0, 1, dca_kernel<4, 8, 16, true, false, 1>, nullptr, 4, "dca_kernel<4, 8, 16, true, false, 1>"},
    {5, 8, 16, 1, 1, 0, 1, dca_kernel<5, 8, 16, true, false, 1>, nullptr, 4, "dca_kernel<5, 8, 16, true, false, 1>"},
    {3, 8, 32, 1, 1, 0, 1, dca_kernel<3, 8, 32, true, false, 1>, nullptr, 4, "dca_kernel<3, 8, 32, true, false, 1>"},
    {4, 16, 32, 1, 1, 0, 1, dca_kernel<4, 16, 32, true, false, 1>, nullptr, 4, "dca_kernel<4, 16, 32, true, false, 1>"},
    {3, 16, 32, 1, 1, 0, 1, dca_kernel<3, 16, 32, true, false, 1>, nullptr, 4, "dca_kernel<3, 16, 32, true, false, 1>"},
    // every wave on its own (no LDS staging)
    {4, 8, 16, 1, 1, 1, 1, dca_kernel<4, 8, 16, true, true, 1>, nullptr, 4, "dca_kernel<4, 8, 16, true, true, 1>"},
    {3, 8, 16, 1, 1, 1, 1, dca_kernel<3, 8, 16, true, true, 1>, nullptr, 4, "dca_kernel<3, 8, 16, true, true, 1>"},
    {2, 8, 16, 1, 1, 1, 1, dca_kernel<2, 8, 16, true, true, 1>, nullptr, 4, "dca_kernel<2, 8, 16, true, true, 1>"},
    {4, 4, 16, 1, 1, 1, 1, dca_kernel<4, 4, 16, true, true, 1>, nullptr, 4, "dca_kernel<4, 4, 16, true, true, 1>"},
    {3, 4, 16, 1, 1, 1, 1, dca_kernel<3, 4, 16, true, true, 1>, nullptr, 4, "dca_kernel<3, 4, 16, true, true, 1>"},
    {4, 8, 32, 1, 1, 1, 1, dca_kernel<4, 8, 32, true, true, 1>, nullptr, 4, "dca_kernel<4, 8, 32, true, true, 1>"},
    // runs of 4 chunks tested first (two-level distance bound)
    {4, 4, 16, 1, 1, 1, 4, dca_kernel<4, 4, 16, true, true, 4>, nullptr, 4, "dca_kernel<4, 4, 16, true, true, 4>"},
    {3, 4, 16, 1, 1, 1, 4, dca_kernel<3, 4, 16, true, true, 4>, nullptr, 4, "dca_kernel<3, 4, 16, true, true, 4>"},
    {4, 8, 16, 1, 1, 1, 4, dca_kernel<4, 8, 16, true, true, 4>, nullptr, 4, "dca_kernel<4, 8, 16, true, true, 4>"},
    {4, 4, 16, 1, 1, 1, 2, dca_kernel<4, 4, 16, true, true, 2>, nullptr, 4, "dca_kernel<4, 4, 16, true, true, 2>"},
    // wide: up to 16 wires per wave in azimuth order, frames in LDS, per-wire skips
    {16, 1, 16, 1, 1, 2, 4, nullptr, dca_wide_kernel<16, 1, 4, 2>, 2, "dca_wide_kernel<16, 1, 4, 2, 0, false>"},
    {16, 2, 16, 1, 1, 2, 4, nullptr, dca_wide_kernel<16, 2, 4, 2>, 2, "dca_wide_kernel<16, 2, 4, 2, 0, false>"},
    {16, 1, 16, 1, 1, 2, 1, nullptr, dca_wide_kernel<16, 1, 1, 2>, 2, "dca_wide_kernel<16, 1, 1, 2, 0, false>"},
    {8, 1, 16, 1, 1, 2, 4, nullptr, dca_wide_kernel<8, 1, 4, 2>, 2, "dca_wide_kernel<8, 1, 4, 2, 0, false>"},
    {16, 4, 16, 1, 1, 2, 4, nullptr, dca_wide_kernel<16, 4, 4, 2>, 2, "dca_wide_kernel<16, 4, 4, 2, 0, false>"},
    {12, 1, 16, 1, 1, 2, 4, nullptr, dca_wide_kernel<12, 1, 4, 2>, 2, "dca_wide_kernel<12, 1, 4, 2, 0, false>"},
    // wide with the chunk tests in batches of 8 or 16 and double-buffered half chunks
    // (runs reports the batch: its first point is tested with the batch's summed radii)
    {8, 1, 16, 1, 1, 2, 8, nullptr, dca_wide_kernel<8, 1, 0, 2, 8>, 2, "dca_wide_kernel<8, 1, 0, 2, 8, false>"},
    {8, 1, 16, 1, 1, 2, 16, nullptr, dca_wide_kernel<8, 1, 0, 2, 16>, 2, "dca_wide_kernel<8, 1, 0, 2, 16, false>"},
    {12, 1, 16, 1, 1, 2, 8, nullptr, dca_wide_kernel<12, 1, 0, 2, 8>, 2, "dca_wide_kernel<12, 1, 0, 2, 8, false>"},
    {16, 1, 16, 1, 1, 2, 8, nullptr, dca_wide_kernel<16, 1, 0, 2, 8>, 2, "dca_wide_kernel<16, 1, 0, 2, 8, false>"},
    {6, 1, 16, 1, 1, 2, 8, nullptr, dca_wide_kernel<6, 1, 0, 3, 8>, 3, "dca_wide_kernel<6, 1, 0, 3, 8, false>"},
    {4, 1, 16, 1, 1, 2, 8, nullptr, dca_wide_kernel<4, 1, 0, 3, 8>, 3, "dca_wide_kernel<4, 1, 0, 3, 8, false>"},
    // wide with the residual cap in the bound (no upper-bound pass; direct == 3)
    {16, 1, 16, 1, 1, 3, 4, nullptr, dca_wide_kernel<16, 1, 4, 2, 0, true>, 2, "dca_wide_kernel<16, 1, 4, 2, 0, true>"},
    {12, 1, 16, 1, 1, 3, 4, nullptr, dca_wide_kernel<12, 1, 4, 2, 0, true>, 2, "dca_wide_kernel<12, 1, 4, 2, 0, true>"},
    {8, 1, 16, 1, 1, 3, 4, nullptr, dca_wide_kernel<8, 1, 4, 2, 0, true>, 2, "dca_wide_kernel<8, 1, 4, 2, 0, true>"},
    {16, 1, 16, 1, 1, 3, 8, nullptr, dca_wide_kernel<16, 1, 0, 2, 8, true>, 2, "dca_wide_kernel<16, 1, 0, 2, 8, true>"},
    {8, 1, 16, 1, 1, 3, 8, nullptr, dca_wide_kernel<8, 1, 0, 2, 8, true>, 2, "dca_wide_kernel<8, 1, 0, 2, 8, true>"},
    {16, 2, 16, 1, 1, 3, 4, nullptr, dca_wide_kernel<16, 2, 4, 2, 0, true>, 2, "dca_wide_kernel<16, 2, 4, 2, 0, true>"},
    // the cap, and the first index of the minimum tracked point by point (direct == 5)
    {16, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<16, 1, 4, 2, 0, true, true>, 2, "dca_wide_kernel<16, 1, 4, 2, 0, true, true>"},
    {12, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<12, 1, 4, 2, 0, true, true>, 2, "dca_wide_kernel<12, 1, 4, 2, 0, true, true>"},
    {8, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<8, 1, 4, 2, 0, true, true>, 2, "dca_wide_kernel<8, 1, 4, 2, 0, true, true>"},
    // ... with each half (or quarter) of a needed chunk tested per wire (within 7 (3) longest
    // steps of its first point)
    {16, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<16, 1, 4, 2, 0, true, true, 2>, 2, "dca_wide_kernel<16, 1, 4, 2, 0, true, true, 2>"},
    {12, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<12, 1, 4, 2, 0, true, true, 2>, 2, "dca_wide_kernel<12, 1, 4, 2, 0, true, true, 2>"},
    {16, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<16, 1, 4, 2, 0, true, true, 4>, 2, "dca_wide_kernel<16, 1, 4, 2, 0, true, true, 4>"},
    {12, 1, 16, 0, 1, 5, 4, nullptr, dca_wide_kernel<12, 1, 4, 2, 0, true, true, 4>, 2, "dca_wide_kernel<12, 1, 4, 2, 0, true, true, 4>"},
};
constexpr int kNumDcaVariants = sizeof(kDcaVariants) / sizeof(kDcaVariants[0]);
constexpr int kMaxWiresPerGroup = 96;  // largest W * NWV in the table above

// Variant choice: an explicit process-wide override, else the autotuned choice for
// the call's shape, else variant 0.
struct ShapeKey {
    int64_t S;
    int P, n_w;
    bool operator<(const ShapeKey &o) const
    {
        return S != o.S ? S < o.S : (P != o.P ? P < o.P : n_w < o.n_w);
    }
};
std::mutex g_tune_mu;
std::map<ShapeKey, int> g_tuned;
int g_dca_variant = -1;  // explicit override; -1 = tuned or default

// Frames are padded so that any variant's last wire group stays in bounds:
// n_groups * (W * NWV) <= n_w + (W * NWV) - 1 <= wire_pad(n_w).
int wire_pad(int n_w)
{
    return ((n_w + 63) / 64) * 64 + kMaxWiresPerGroup;
}

size_t frames_region_bytes(int n_w)
{
    const size_t pad = (size_t)wire_pad(n_w);
    return 2 * align256(sizeof(double) * 8 * pad) + 2 * align256(sizeof(int32_t) * pad) +
           align256(sizeof(double) * pad);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int comet_version(void) { return kVersion; }

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
    clear_error();
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
    clear_error();
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
    clear_error();
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
                       cfg->charge_e, cfg->step_mm, cfg->n_steps, track_xyz, (double *)nullptr);
    return launched("rk4_record_kernel");
}

size_t comet_dca_workspace_bytes(int64_t n_seeds, int32_t n_points, int32_t n_wires)
{
    if (n_seeds < 1 || n_points < 1 || n_wires < 0)
        return 0;
    return frames_region_bytes(n_wires) +
           align256(sizeof(double) * (size_t)n_wires * (size_t)n_seeds) +
           align256(sizeof(double) * (size_t)cdev::radius_rows(n_points) * (size_t)n_seeds);
}

}  // extern "C"

namespace {

// Host-side checks shared by comet_dca_rss and comet_dca_autotune.
int check_dca_args(const char *who, const double *track_xyz, int64_t n_seeds, int32_t n_points,
                   const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                   const double *drift, int32_t n_hits, const comet_config *cfg, const double *rss,
                   const void *workspace, size_t workspace_bytes)
{
    if (!track_xyz || !rss)
        return fail(COMET_EINVAL, "%s: NULL pointer", who);
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "%s: n_seeds = %lld", who, (long long)n_seeds);
    if (n_wires < 0 || n_hits < 0)
        return fail(COMET_EINVAL, "%s: negative n_wires or n_hits", who);
    if (n_wires > 0 && (!wire_ends || !wire_offsets || (n_hits > 0 && !drift)))
        return fail(COMET_EINVAL, "%s: NULL wire or hit array", who);
    int st = check_config(cfg);
    if (st)
        return st;
    if (n_points != cfg->n_steps + 1)
        return fail(COMET_EINVAL, "%s: n_points %d != n_steps + 1", who, n_points);
    if ((int64_t)(n_seeds + 63) / 64 * (int64_t)((n_wires + 15) / 16) > (int64_t)1 << 30)
        return fail(COMET_EINVAL, "%s: problem too large for one launch", who);
    if (n_wires > 0) {
        const size_t need = comet_dca_workspace_bytes(n_seeds, n_points, n_wires);
        if (!workspace || workspace_bytes < need)
            return fail(COMET_EWORKSPACE, "%s: workspace %zu < %zu bytes", who, workspace_bytes,
                        need);
        if (((uintptr_t)workspace & 255) != 0)
            return fail(COMET_EINVAL, "%s: workspace not 256-byte aligned", who);
    }
    return COMET_OK;
}

// The workspace: frames in wire order, frames in azimuth order, each azimuth slot's
// wire, each azimuth slot's cap (the wire's largest drift distance, -1 without hits),
// the azimuth keys (together frames_region_bytes), then dsq[n_w][S], then the chunk
// radii [radius_chunks(P)][S] followed by each track's longest step [S].
double *dca_frames(void *workspace) { return (double *)workspace; }

double *dca_frames_sorted(void *workspace, int n_wires)
{
    return (double *)((char *)workspace + align256(sizeof(double) * 8 * (size_t)wire_pad(n_wires)));
}

int32_t *dca_wire_of(void *workspace, int n_wires)
{
    return (int32_t *)((char *)workspace +
                       2 * align256(sizeof(double) * 8 * (size_t)wire_pad(n_wires)));
}

float *dca_keys(void *workspace, int n_wires)
{
    return (float *)((char *)dca_wire_of(workspace, n_wires) +
                     align256(sizeof(int32_t) * (size_t)wire_pad(n_wires)));
}

double *dca_caps(void *workspace, int n_wires)
{
    return (double *)((char *)dca_keys(workspace, n_wires) +
                      align256(sizeof(float) * (size_t)wire_pad(n_wires)));
}

double *dca_dsq(void *workspace, int n_wires)
{
    return (double *)((char *)workspace + frames_region_bytes(n_wires));
}

double *dca_rho(void *workspace, int n_wires, int64_t n_seeds)
{
    return (double *)((char *)dca_dsq(workspace, n_wires) +
                      align256(sizeof(double) * (size_t)n_wires * (size_t)n_seeds));
}

int launch_radius(const double *track_xyz, int64_t n_seeds, int32_t n_points, int n_wires,
                  void *workspace, hipStream_t hs)
{
    // the longest-step row starts at 0 (the radius kernel raises it with atomicMax)
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                       dca_rho(workspace, n_wires, n_seeds) +
                           (int64_t)cdev::radius_chunks(n_points) * n_seeds,
                       n_seeds, 0.0);
    int st = launched("fill_kernel");
    if (st)
        return st;
    hipLaunchKernelGGL(chunk_radius_kernel,
                       dim3((unsigned)((n_seeds + 255) / 256),
                            (unsigned)std::min(cdev::radius_chunks(n_points), 65535)),
                       dim3(256), 0, hs, track_xyz, n_seeds, n_points,
                       dca_rho(workspace, n_wires, n_seeds));
    return launched("chunk_radius_kernel");
}

int launch_frames(const double *wire_ends, int n_wires, const int32_t *wire_offsets,
                  const double *drift, void *workspace, hipStream_t hs)
{
    const int pad = wire_pad(n_wires);
    hipLaunchKernelGGL(frame_kernel, dim3((pad + 63) / 64), dim3(64), 0, hs, wire_ends, n_wires,
                       pad, dca_frames(workspace), dca_keys(workspace, n_wires));
    int st = launched("frame_kernel");
    if (st)
        return st;
    hipLaunchKernelGGL(wire_order_kernel, dim3((pad + 255) / 256), dim3(256), 0, hs,
                       (const double *)dca_frames(workspace),
                       (const float *)dca_keys(workspace, n_wires), pad, n_wires, wire_offsets,
                       drift, dca_frames_sorted(workspace, n_wires), dca_wire_of(workspace, n_wires),
                       dca_caps(workspace, n_wires));
    return launched("wire_order_kernel");
}

int launch_dca(int id, const double *track_xyz, int64_t n_seeds, int32_t n_points, int n_wires,
               const int32_t *wire_offsets, const double *drift, double lambda, void *workspace,
               hipStream_t hs)
{
    const DcaVariant &v = kDcaVariants[id];
    const int per_group = v.w * v.nwv;
    const int n_groups = (n_wires + per_group - 1) / per_group;
    const int64_t n_tiles = (n_seeds + 63) / 64;
    const int64_t n_blocks = n_tiles * n_groups;
    if (v.wide) {
        hipLaunchKernelGGL(v.wide, dim3((unsigned)n_blocks), dim3(64 * v.nwv), 0, hs, track_xyz,
                           n_seeds, n_points, (const double *)dca_frames_sorted(workspace, n_wires),
                           (const int32_t *)dca_wire_of(workspace, n_wires),
                           (const double *)dca_caps(workspace, n_wires), n_wires, wire_offsets,
                           drift, lambda, (const double *)dca_rho(workspace, n_wires, n_seeds),
                           dca_dsq(workspace, n_wires), n_groups, (int)n_blocks, v.xcd_remap,
                           scan_counter());
        return launched("dca_wide_kernel");
    }
    hipLaunchKernelGGL(v.kernel, dim3((unsigned)n_blocks), dim3(64 * v.nwv), 0, hs, track_xyz,
                       n_seeds, n_points, (const double *)dca_frames(workspace), n_wires,
                       wire_offsets, drift, lambda,
                       (const double *)dca_rho(workspace, n_wires, n_seeds),
                       dca_dsq(workspace, n_wires), n_groups, (int)n_blocks, v.xcd_remap,
                       scan_counter());
    return launched("dca_kernel");
}

int choose_variant(int64_t S, int P, int n_w)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_dca_variant >= 0)
        return g_dca_variant;
    auto it = g_tuned.find(ShapeKey{S, P, n_w});
    return it == g_tuned.end() ? 0 : it->second;
}

}  // namespace

extern "C" {

int comet_dca_rss(const double *track_xyz, int64_t n_seeds, int32_t n_points,
                  const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                  const double *drift, int32_t n_hits, const comet_config *cfg, double *rss,
                  void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    int st = check_dca_args("comet_dca_rss", track_xyz, n_seeds, n_points, wire_ends, n_wires,
                            wire_offsets, drift, n_hits, cfg, rss, workspace, workspace_bytes);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    if (n_wires == 0) {
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                           rss, n_seeds, 0.0);
        return launched("fill_kernel");
    }
    st = launch_frames(wire_ends, n_wires, wire_offsets, drift, workspace, hs);
    if (st)
        return st;
    st = launch_radius(track_xyz, n_seeds, n_points, n_wires, workspace, hs);
    if (st)
        return st;
    {
        ProfScope prof(kProfDca, hs);
        st = launch_dca(choose_variant(n_seeds, n_points, n_wires), track_xyz, n_seeds, n_points,
                        n_wires, wire_offsets, drift, cfg->lambda_mm, workspace, hs);
    }
    if (st)
        return st;
    ProfScope prof(kProfSum, hs);
    hipLaunchKernelGGL(rss_sum_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                       (const double *)dca_dsq(workspace, n_wires), n_wires, n_seeds, rss);
    return launched("rss_sum_kernel");
}

}  // extern "C"

namespace {

// The body of comet_track_dca_rss and comet_track_dca_rss_static (arguments checked).
int track_dca_rss(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                  const comet_field *field, const double *wire_ends, int32_t n_wires,
                  const int32_t *wire_offsets, const double *drift, double *track_xyz,
                  double *rss, void *workspace, void *stream, bool timed)
{
    int st = COMET_OK;
    hipStream_t hs = (hipStream_t)stream;
    const int P = cfg->n_steps + 1;
    double *rho = n_wires > 0 ? dca_rho(workspace, n_wires, n_seeds) : nullptr;
    {
        ProfScope prof(kProfTrack, hs, timed);
        if (field) {
            st = launch_field_record(seeds6, n_seeds, field, cfg->charge_e, cfg->step_mm,
                                     cfg->n_steps, track_xyz, rho, hs);
        } else {
            const int threads = 256;
            hipLaunchKernelGGL(rk4_record_kernel,
                               dim3((unsigned)((n_seeds + threads - 1) / threads)), dim3(threads),
                               0, hs, seeds6, n_seeds, cfg->bz_tesla, cfg->charge_e,
                               cfg->step_mm, cfg->n_steps, track_xyz, rho);
            st = launched("rk4_record_kernel");
        }
    }
    if (st)
        return st;
    if (n_wires == 0) {
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                           rss, n_seeds, 0.0);
        return launched("fill_kernel");
    }
    st = launch_frames(wire_ends, n_wires, wire_offsets, drift, workspace, hs);
    if (st)
        return st;
    {
        ProfScope prof(kProfDca, hs, timed);
        st = launch_dca(choose_variant(n_seeds, P, n_wires), track_xyz, n_seeds, P, n_wires,
                        wire_offsets, drift, cfg->lambda_mm, workspace, hs);
    }
    if (st)
        return st;
    ProfScope prof(kProfSum, hs, timed);
    hipLaunchKernelGGL(rss_sum_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                       (const double *)dca_dsq(workspace, n_wires), n_wires, n_seeds, rss);
    return launched("rss_sum_kernel");
}

int check_track_dca_args(const char *who, const double *seeds6, int64_t n_seeds,
                         const comet_config *cfg, const comet_field *field,
                         const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                         const double *drift, int32_t n_hits, double *track_xyz, double *rss,
                         void *workspace, size_t workspace_bytes)
{
    if (!seeds6)
        return fail(COMET_EINVAL, "%s: NULL seeds", who);
    int st = check_dca_args(who, track_xyz, n_seeds, cfg ? cfg->n_steps + 1 : 0, wire_ends,
                            n_wires, wire_offsets, drift, n_hits, cfg, rss, workspace,
                            workspace_bytes);
    if (st)
        return st;
    if (field) {
        st = check_field(who, field);
        if (st)
            return st;
    }
    return check_device();
}

// The workspace of comet_track_dca_rss_static: a fixed array in device memory, one
// copy per GPU, for callers that cannot allocate. Its host-side name is not a device
// address; each device's address comes from hipGetSymbolAddress on the first call
// made with that device current.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

int static_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(COMET_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64)
        return fail(COMET_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(COMET_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return COMET_OK;
}

}  // namespace

extern "C" {

int comet_track_dca_rss(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                        const comet_field *field, const double *wire_ends, int32_t n_wires,
                        const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                        double *track_xyz, double *rss, void *workspace, size_t workspace_bytes,
                        void *stream)
{
    clear_error();
    const int st = check_track_dca_args("comet_track_dca_rss", seeds6, n_seeds, cfg, field,
                                        wire_ends, n_wires, wire_offsets, drift, n_hits, track_xyz,
                                        rss, workspace, workspace_bytes);
    if (st)
        return st;
    return track_dca_rss(seeds6, n_seeds, cfg, field, wire_ends, n_wires, wire_offsets, drift,
                         track_xyz, rss, workspace, stream, true);
}

size_t comet_static_scratch_bytes(void) { return kStaticScratchBytes; }

int comet_track_dca_rss_static(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                               const comet_field *field, const double *wire_ends,
                               int32_t n_wires, const int32_t *wire_offsets, const double *drift,
                               int32_t n_hits, double *track_xyz, double *rss, void *stream)
{
    clear_error();
    const int P = cfg ? cfg->n_steps + 1 : 0;
    if (n_seeds >= 1 && P >= 1 && n_wires >= 0 &&
        comet_dca_workspace_bytes(n_seeds, P, n_wires) > kStaticScratchBytes)
        return fail(COMET_EWORKSPACE,
                    "comet_track_dca_rss_static: %lld seeds x %d points x %d wires need %zu bytes "
                    "of workspace, more than the fixed %zu (split the seeds)",
                    (long long)n_seeds, P, n_wires, comet_dca_workspace_bytes(n_seeds, P, n_wires),
                    kStaticScratchBytes);
    // the arguments first (the array's address stands in until it is known), then the
    // array's address on the current device
    int st = check_track_dca_args("comet_track_dca_rss_static", seeds6, n_seeds, cfg, field,
                                  wire_ends, n_wires, wire_offsets, drift, n_hits, track_xyz, rss,
                                  (void *)256, kStaticScratchBytes);
    if (st)
        return st;
    void *ws = nullptr;
    st = static_scratch(&ws);
    if (st)
        return st;
    // no event timing here: the profiler's events are created on demand
    return track_dca_rss(seeds6, n_seeds, cfg, field, wire_ends, n_wires, wire_offsets, drift,
                         track_xyz, rss, ws, stream, false);
}

int comet_dca_autotune(const double *track_xyz, int64_t n_seeds, int32_t n_points,
                       const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                       const double *drift, int32_t n_hits, const comet_config *cfg, double *rss,
                       void *workspace, size_t workspace_bytes, int32_t reps, int32_t *best_id,
                       double *ms, void *stream)
{
    clear_error();
    int st = check_dca_args("comet_dca_autotune", track_xyz, n_seeds, n_points, wire_ends,
                            n_wires, wire_offsets, drift, n_hits, cfg, rss, workspace,
                            workspace_bytes);
    if (st)
        return st;
    if (reps < 1 || reps > 1000)
        return fail(COMET_EINVAL, "comet_dca_autotune: reps must be in [1, 1000]");
    if (n_wires == 0)
        return fail(COMET_EINVAL, "comet_dca_autotune: nothing to tune without wires");
    st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    st = launch_frames(wire_ends, n_wires, wire_offsets, drift, workspace, hs);
    if (st)
        return st;
    st = launch_radius(track_xyz, n_seeds, n_points, n_wires, workspace, hs);
    if (st)
        return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return fail(COMET_EHIP, "comet_dca_autotune: hipEventCreate failed");
    }
    int best = -1;
    float best_ms = 0.0f;
    float times[kNumDcaVariants];
    for (int id = 0; id < kNumDcaVariants && st == COMET_OK; ++id) {
        st = launch_dca(id, track_xyz, n_seeds, n_points, n_wires, wire_offsets, drift,
                        cfg->lambda_mm, workspace, hs);  // warm-up
        (void)hipEventRecord(e0, hs);
        for (int r = 0; r < reps && st == COMET_OK; ++r)
            st = launch_dca(id, track_xyz, n_seeds, n_points, n_wires, wire_offsets, drift,
                            cfg->lambda_mm, workspace, hs);
        (void)hipEventRecord(e1, hs);
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess && st == COMET_OK)
            st = fail(COMET_EHIP, "comet_dca_autotune: %s", hipGetErrorString(e));
        t /= (float)reps;
        times[id] = t;
        if (ms)
            ms[id] = t;
        if (st == COMET_OK && (best < 0 || t < best_ms)) {
            best = id;
            best_ms = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st)
        return st;
    // Within 1 % of the fastest, prefer fewer wire groups: each group reads the seed
    // tile's track again, so fewer groups means less memory traffic at equal speed.
    {
        auto groups = [&](int id) {
            const int g = kDcaVariants[id].w * kDcaVariants[id].nwv;
            return (n_wires + g - 1) / g;
        };
        int pick = best;
        for (int id = 0; id < kNumDcaVariants; ++id) {
            if (times[id] <= 1.01f * best_ms &&
                (groups(id) < groups(pick) || (groups(id) == groups(pick) && times[id] < times[pick])))
                pick = id;
        }
        best = pick;
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[ShapeKey{n_seeds, n_points, n_wires}] = best;
    }
    if (best_id)
        *best_id = best;
    // leave rss consistent with the inputs
    hipLaunchKernelGGL(rss_sum_kernel, dim3((unsigned)((n_seeds + 255) / 256)), dim3(256), 0, hs,
                       (const double *)dca_dsq(workspace, n_wires), n_wires, n_seeds, rss);
    return launched("rss_sum_kernel");
}

int comet_select_classify(const double *rss, int64_t n_seeds, const double *track_xyz,
                          int32_t n_points, const double *wire_ends, int32_t n_wires,
                          const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                          const comet_config *cfg, int32_t top_k, int64_t *best,
                          uint8_t *hit_mask, int32_t *n_borderline, double *dca_best,
                          void *stream)
{
    clear_error();
    if (!rss || !best)
        return fail(COMET_EINVAL, "comet_select_classify: NULL rss or best");
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "comet_select_classify: n_seeds = %lld", (long long)n_seeds);
    if (top_k < 1 || top_k > 1024)
        return fail(COMET_EINVAL, "comet_select_classify: top_k must be in [1, 1024]");
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
    if (top_k > 1) {
        st = comet_topk(rss, n_seeds, 1, top_k, best, stream);
        if (st)
            return st;
    }
    ProfScope prof(kProfSelect, hs);
    if (top_k == 1) {
        hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(kSelectThreads), 0, hs, rss, n_seeds,
                           best);
        st = launched("argmin_kernel");
    }
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
                           int32_t *chunk_argmin, int32_t *xcd_remap, int32_t *direct,
                           int32_t *runs)
{
    if (id < 0 || id >= kNumDcaVariants || !w || !nwv || !chunk || !chunk_argmin || !xcd_remap)
        return fail(COMET_EINVAL, "comet_dca_variant_info: bad id or NULL pointer");
    *w = kDcaVariants[id].w;
    *nwv = kDcaVariants[id].nwv;
    *chunk = kDcaVariants[id].c;
    *chunk_argmin = kDcaVariants[id].chunk_argmin;
    *xcd_remap = kDcaVariants[id].xcd_remap;
    if (direct)
        *direct = kDcaVariants[id].direct;
    if (runs)
        *runs = kDcaVariants[id].sup;
    return COMET_OK;
}

const char *comet_dca_variant_name(int id)
{
    if (id < 0 || id >= kNumDcaVariants)
        return "";
    return kDcaVariants[id].name;
}

int comet_dca_set_variant(int id)
{
    if (id < -1 || id >= kNumDcaVariants)
        return fail(COMET_EINVAL, "comet_dca_set_variant: id %d out of range", id);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_dca_variant = id;
    return COMET_OK;
}

int comet_dca_variant_for(int64_t n_seeds, int32_t n_points, int32_t n_wires)
{
    return choose_variant(n_seeds, n_points, n_wires);
}

}  // extern "C"
