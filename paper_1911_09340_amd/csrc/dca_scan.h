// dca_scan.h -- the DCA / Eq. 1 scan of one 64-seed tile against a block's wires,
// shared by the single-event kernel (comet.hip) and the batched persistent kernel
// (batch.hip), so that both produce the same bits.
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 2.2.2 (Alg. 2) and Eq. 1.
//
// Layout: coordinate c of track point k for tile lane l sits at base_c[k * ld + l]
// (base_x, base_y, base_z; lanes l < n_valid hold seeds). Each of the block's NWV
// waves owns W wires whose frames are in registers (`f`). The tile's track streams
// through LDS in chunks of C points, loaded once per block and read by every wave.
// Two LDS buffers alternate: while the waves scan chunk n from one, chunk n + 1 is
// stored into the other from registers, and chunk n + 2 is already being loaded
// from memory, so one barrier per chunk suffices.
//
// Every lane keeps, per wire, the smallest q = xi^2 + eta^2 seen so far and the first
// index reaching it (Alg. 2: the recorded state closest to the wire); the index is
// either tracked per point (CHUNK_ARGMIN = false) or per chunk (true: a running min
// per point, the chunk holding the first minimum recorded, and that chunk rescanned
// from memory at the end with the same arithmetic, so equality finds the first
// index). The closest point is then refined over its two chords and Eq. 1's capped
// residual d = min(lambda, min_j |D - r_j|) is formed.
#ifndef COMET_DCA_SCAN_H
#define COMET_DCA_SCAN_H

#include "device_math.h"

namespace cdev {

template <int W, int NWV, int C, bool CHUNK_ARGMIN>
struct TileScan {
    static constexpr int kChunkDoubles = 3 * C * 64;
    static constexpr int kLdsDoubles = 2 * kChunkDoubles;

    // Returns d^2 of (lane, wire w) in dsq[w] for lanes < n_valid and w < nw (0
    // elsewhere). nw (this wave's wire count, 0..W) must be wave-uniform; offsets
    // points at the CSR entry of the wave's first wire. Every thread of the block
    // must call this (it synchronises the block); lds holds kLdsDoubles doubles.
    __device__ static void run(const double *__restrict__ bx, const double *__restrict__ by,
                               const double *__restrict__ bz, int64_t ld, int P, int n_valid,
                               bool pairs, const double (&f)[W][8], int nw,
                               const int32_t *__restrict__ offsets,
                               const double *__restrict__ drift, double lambda,
                               double *__restrict__ lds, double (&dsq)[W])
    {
        const int lane = threadIdx.x & 63;
        const bool active = nw > 0;
        double best[W], cmin[W];
        int kbest[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            best[w] = INFINITY;
            kbest[w] = 0;
        }

        // Each thread owns PER_T slots of two consecutive lanes (16 bytes).
        constexpr int T = 64 * NWV;
        constexpr int UNITS = 3 * C * 32;
        constexpr int PER_T = (UNITS + T - 1) / T;
        const bool full_tile = pairs && n_valid == 64;
        double2 pre[PER_T];
        auto fetch = [&](int k0) {
            if (full_tile && k0 + C <= P) {
                // whole chunk in range, every lane a seed: plain 16-byte loads
#pragma unroll
                for (int u = 0; u < PER_T; ++u) {
                    const int idx = threadIdx.x + u * T;
                    if (UNITS % T == 0 || idx < UNITS) {
                        const int c = idx / (C * 32);
                        const int r = idx - c * (C * 32);
                        const double *src = (c == 0 ? bx : (c == 1 ? by : bz)) +
                                            (int64_t)(k0 + (r >> 5)) * ld + (r & 31) * 2;
                        pre[u] = *reinterpret_cast<const double2 *>(src);
                    }
                }
                return;
            }
#pragma unroll
            for (int u = 0; u < PER_T; ++u) {
                const int idx = threadIdx.x + u * T;
                const int c = idx / (C * 32);
                const int r = idx - c * (C * 32);
                const int kk = r >> 5;
                const int l2 = (r & 31) * 2;
                const int k = k0 + kk;
                double2 v = make_double2(0.0, 0.0);
                if (idx < UNITS && k < P) {
                    const double *src = (c == 0 ? bx : (c == 1 ? by : bz)) + (int64_t)k * ld + l2;
                    if (pairs && l2 + 1 < n_valid) {
                        v = *reinterpret_cast<const double2 *>(src);
                    } else {
                        if (l2 < n_valid)
                            v.x = src[0];
                        if (l2 + 1 < n_valid)
                            v.y = src[1];
                    }
                }
                pre[u] = v;
            }
        };
        auto stash = [&](double *buf) {
#pragma unroll
            for (int u = 0; u < PER_T; ++u) {
                const int idx = threadIdx.x + u * T;
                if (UNITS % T == 0 || idx < UNITS)
                    *reinterpret_cast<double2 *>(&buf[2 * idx]) = pre[u];
            }
        };
        auto point = [&](const double *buf, int kk, int k, bool first) {
            const double x = buf[(0 * C + kk) * 64 + lane];
            const double y = buf[(1 * C + kk) * 64 + lane];
            const double z = buf[(2 * C + kk) * 64 + lane];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double xi, eta;
                project(f[w], x, y, z, xi, eta);
                const double q = fma(xi, xi, eta * eta);
                if (CHUNK_ARGMIN) {
                    cmin[w] = first ? q : fmin(cmin[w], q);
                } else {
                    kbest[w] = q < best[w] ? k : kbest[w];
                    best[w] = fmin(best[w], q);
                }
            }
        };

        // prologue: chunk 0 into buffer 0, chunk 1 in flight
        fetch(0);
        __syncthreads();  // the previous caller's reads of lds are done
        stash(lds);
        if (C < P)
            fetch(C);
        __syncthreads();

        for (int k0 = 0, n = 0; k0 < P; k0 += C, ++n) {
            const double *cur = lds + (n & 1) * kChunkDoubles;
            if (active) {
                const int kn = min(C, P - k0);
                if (kn == C) {
#pragma unroll
                    for (int kk = 0; kk < C; ++kk)
                        point(cur, kk, k0 + kk, kk == 0);
                } else {
                    point(cur, 0, k0, true);
                    for (int kk = 1; kk < kn; ++kk)
                        point(cur, kk, k0 + kk, false);
                }
                if (CHUNK_ARGMIN) {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        if (cmin[w] < best[w]) {
                            best[w] = cmin[w];
                            kbest[w] = k0;
                        }
                    }
                }
            }
            if (k0 + C < P) {
                // chunk n + 1 goes to the other buffer, whose chunk n - 1 every wave
                // finished before the previous barrier
                stash(lds + ((n + 1) & 1) * kChunkDoubles);
                if (k0 + 2 * C < P)
                    fetch(k0 + 2 * C);
            }
            __syncthreads();
        }

#pragma unroll
        for (int w = 0; w < W; ++w)
            dsq[w] = 0.0;
        if (!active || lane >= n_valid)
            return;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (w < nw) {
                int k = kbest[w];
                if (CHUNK_ARGMIN) {
                    const int kend = min(k + C, P);
                    int kf = k;
                    for (int j = k; j < kend; ++j) {
                        const int64_t o = (int64_t)j * ld + lane;
                        double xi, eta;
                        project(f[w], bx[o], by[o], bz[o], xi, eta);
                        if (fma(xi, xi, eta * eta) == best[w]) {
                            kf = j;
                            break;
                        }
                    }
                    k = kf;
                }
                const double d2 = refine_dca2(bx + lane, by + lane, bz + lane, ld, P, f[w], k,
                                              best[w]);
                const double D = sqrt(d2);
                const double d = capped_residual(D, drift, offsets[w], offsets[w + 1], lambda);
                dsq[w] = d * d;
            }
        }
    }
};

}  // namespace cdev

#endif  // COMET_DCA_SCAN_H
