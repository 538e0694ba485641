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
//
// Distance bound (exact; it only saves work). Every point of a chunk lies within rho
// (the chunk radius, ChunkRadius in device_math.h) of the chunk's first point p0, so
// its distance to a wire is at least dist(p0) - rho. (A) The first points of every
// other chunk give each (lane, wire) an upper bound ub of its final minimum q. (B) A wave
// needs a chunk unless, for every lane and every wire it owns, sqrt(q(p0)) exceeds
// rho + sqrt(ub) (with margins far above the rounding of either side): then no point
// of the chunk can reach or tie the final minimum. (C) Only the chunks some wave of
// the block needs go through LDS, and each wave scans only the ones it needs. The
// chunk holding the first minimum is always scanned, so the minimum, its first index
// and every result are those of the full scan. Chunks are handled in segments of 256
// (any track length).
#ifndef COMET_DCA_SCAN_H
#define COMET_DCA_SCAN_H

#include "device_math.h"

namespace cdev {

// The end of a tile scan (both forms below): the evaluation count, then per (lane,
// wire) the first index of the minimum (per chunk: rescan the chunk that holds it),
// its chord refinement, D and Eq. 1's capped residual.
template <int W, int C, bool CHUNK_ARGMIN>
__device__ __forceinline__ void scan_finish(const double *__restrict__ bx,
                                            const double *__restrict__ by,
                                            const double *__restrict__ bz, int64_t ld, int P,
                                            int n_valid, const double (&f)[W][8], int nw,
                                            const int32_t *__restrict__ offsets,
                                            const double *__restrict__ drift, double lambda,
                                            unsigned long long *counter, int64_t evals,
                                            const double (&best)[W], const int (&kbest)[W],
                                            double (&dsq)[W])
{
    const int lane = threadIdx.x & 63;
    if (counter && lane == 0 && evals > 0)
        atomicAdd(counter, (unsigned long long)(evals * n_valid));
#pragma unroll
    for (int w = 0; w < W; ++w)
        dsq[w] = 0.0;
    if (nw <= 0 || lane >= n_valid)
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
            const double d2 =
                refine_dca2(bx + lane, by + lane, bz + lane, ld, P, f[w], k, best[w]);
            const double D = sqrt(d2);
            const double d = capped_residual(D, drift, offsets[w], offsets[w + 1], lambda);
            dsq[w] = d * d;
        }
    }
}

template <int W, int NWV, int C, bool CHUNK_ARGMIN>
struct TileScan {
    static constexpr int kChunkDoubles = 3 * C * 64;
    static constexpr int kSegChunks = 256;  // chunks per segment of the need pass
    static constexpr int kSegWords = kSegChunks / 64;
    // LDS: two chunk buffers, the need bits of every wave for one segment, then the
    // segment's list of needed chunks, the per-wave counts and their total (ints).
    static constexpr int kMaskOffset = 2 * kChunkDoubles;
    static constexpr int kListOffset = kMaskOffset + NWV * kSegWords;
    static constexpr int kLdsDoubles = kListOffset + (kSegChunks + NWV + 2) / 2 + 1;
    static_assert(64 * NWV >= kSegChunks, "one thread per chunk of a segment");

    // Returns d^2 of (lane, wire w) in dsq[w] for lanes < n_valid and w < nw (0
    // elsewhere). nw (this wave's wire count, 0..W) must be wave-uniform; offsets
    // points at the CSR entry of the wave's first wire. Every thread of the block
    // must call this (it synchronises the block); lds holds kLdsDoubles doubles.
    // rho: the tile's chunk radii, window n of lane l at rho[n * ldr + l] (lanes <
    // n_valid are read). counter (may be null): receives the (seed, wire, point)
    // distance evaluations performed.
    __device__ static void run(const double *__restrict__ bx, const double *__restrict__ by,
                               const double *__restrict__ bz, int64_t ld, int P, int n_valid,
                               bool pairs, const double (&f)[W][8], int nw,
                               const int32_t *__restrict__ offsets,
                               const double *__restrict__ drift, double lambda,
                               const double *__restrict__ rho, int64_t ldr,
                               unsigned long long *counter, double *__restrict__ lds,
                               double (&dsq)[W])
    {
        static_assert(C % kRadiusChunk == 0 && C / kRadiusChunk <= 2, "chunk of 16 or 32");
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const bool active = nw > 0;
        const bool seed = lane < n_valid;
        uint64_t *const wmask = reinterpret_cast<uint64_t *>(lds + kMaskOffset);
        int *const list = reinterpret_cast<int *>(lds + kListOffset);
        int *const wtot = list + kSegChunks;
        const int nch = (P + C - 1) / C;
        double best[W], cmin[W];
        float ub[W];  // rounded to nearest: the test's margins cover it
        int kbest[W];
        int64_t evals = 0;  // wave-uniform: distance evaluations per seed lane
#pragma unroll
        for (int w = 0; w < W; ++w) {
            best[w] = INFINITY;
            kbest[w] = 0;
            ub[w] = INFINITY;
        }
        // points k0 + i * stride (i < 4, those below P) of this lane; 0 elsewhere
        constexpr int kGather = 2;
        auto gather = [&](int k0, int stride, double (&x)[kGather], double (&y)[kGather],
                          double (&z)[kGather]) {
#pragma unroll
            for (int i = 0; i < kGather; ++i) {
                const int k = k0 + i * stride;
                x[i] = y[i] = z[i] = 0.0;
                if (seed && k < P) {
                    const int64_t o = (int64_t)k * ld + lane;
                    x[i] = bx[o];
                    y[i] = by[o];
                    z[i] = bz[o];
                }
            }
        };
        // (A) upper bounds of the final minima: every other chunk's first point
        if (active) {
            int n_s = 0;
            for (int k0 = 0; k0 < P; k0 += kGather * 2 * C) {
                double x[kGather], y[kGather], z[kGather];
                gather(k0, 2 * C, x, y, z);
#pragma unroll
                for (int i = 0; i < kGather; ++i) {
                    if (k0 + i * 2 * C < P) {
                        ++n_s;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            double xi, eta;
                            project(f[w], x[i], y[i], z[i], xi, eta);
                            ub[w] = fminf(ub[w], (float)fma(xi, xi, eta * eta));
                        }
                    }
                }
            }
            evals += (int64_t)nw * n_s;
        }
        // sqrt(ub) rounded up (FP32 sqrt is within 1 ulp; the factor covers it)
        float sub[W];
#pragma unroll
        for (int w = 0; w < W; ++w)
            sub[w] = __builtin_amdgcn_sqrtf(ub[w]) * 1.000001f;

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

        for (int s0 = 0; s0 < nch; s0 += kSegChunks) {
            const int sn = min(kSegChunks, nch - s0);
            // (B) this wave's need bit of every chunk of the segment: some lane and wire
            // whose bound does not rule the chunk out (the partial last chunk always)
#pragma unroll 1
            for (int word = 0; word < kSegWords; ++word) {
                uint64_t m = 0;
                if (active) {
#pragma unroll 1
                    for (int b0 = 0; b0 < 64 && word * 64 + b0 < sn; b0 += kGather) {
                        const int kb = (s0 + word * 64 + b0) * C;
                        double x[kGather], y[kGather], z[kGather], r[kGather];
                        gather(kb, C, x, y, z);
#pragma unroll
                        for (int i = 0; i < kGather; ++i) {
                            const int k0 = kb + i * C;
                            r[i] = 0.0;
                            if (seed && k0 + C <= P) {
                                const int nr = k0 / kRadiusChunk;
                                r[i] = rho[(int64_t)nr * ldr + lane];
                                if (C == 2 * kRadiusChunk)
                                    r[i] = r[i] + rho[(int64_t)(nr + 1) * ldr + lane];
                            }
                        }
#pragma unroll
                        for (int i = 0; i < kGather; ++i) {
                            const int b = b0 + i;
                            const int k0 = kb + i * C;
                            if (b >= 64 || word * 64 + b >= sn)
                                break;
                            bool need = true;
                            if (k0 + C <= P) {
                                evals += nw;
                                const float rf = (float)r[i] * 1.000001f;
                                bool lane_need = false;
#pragma unroll
                                for (int w = 0; w < W; ++w) {
                                    if (w < nw) {
                                        double xi, eta;
                                        project(f[w], x[i], y[i], z[i], xi, eta);
                                        const float q0 = (float)fma(xi, xi, eta * eta);
                                        const float B = fmaf(rf + sub[w], 1.000001f, 1e-6f);
                                        lane_need = lane_need ||
                                                    !(q0 * 0.999999f > (B * B) * 1.000001f);
                                    }
                                }
                                need = __builtin_amdgcn_ballot_w64(lane_need && seed) != 0;
                            }
                            if (need)
                                m |= 1ull << b;
                        }
                    }
                }
                if (lane == 0)
                    wmask[wave * kSegWords + word] = m;
            }
            __syncthreads();
            // the segment's needed chunks in order (any wave's bit), one thread per chunk
            const int t = threadIdx.x;
            bool flag = false;
            if (t < sn)
                for (int v = 0; v < NWV; ++v)
                    flag = flag || ((wmask[v * kSegWords + (t >> 6)] >> (t & 63)) & 1);
            const uint64_t bal = __builtin_amdgcn_ballot_w64(flag);
            const int below = __builtin_popcountll(bal & ((1ull << lane) - 1));
            if (lane == 0)
                wtot[wave] = __builtin_popcountll(bal);
            __syncthreads();
            int base = 0, total = 0;
            for (int v = 0; v < NWV; ++v) {
                const int c = wtot[v];
                base += v < wave ? c : 0;
                total += c;
            }
            total = __builtin_amdgcn_readfirstlane(total);
            if (flag)
                list[base + below] = t;
            __syncthreads();
            if (total == 0)
                continue;

            // (C) the needed chunks through LDS: chunk j scanned from one buffer while
            // chunk j + 1 is stored into the other and chunk j + 2 is loaded
            fetch((s0 + list[0]) * C);
            stash(lds);
            if (total > 1)
                fetch((s0 + list[1]) * C);
            __syncthreads();
            for (int j = 0; j < total; ++j) {
                const int n = __builtin_amdgcn_readfirstlane(list[j]);
                const int k0 = (s0 + n) * C;
                const double *cur = lds + (j & 1) * kChunkDoubles;
                const bool mine =
                    __builtin_amdgcn_readfirstlane(
                        (int)((wmask[wave * kSegWords + (n >> 6)] >> (n & 63)) & 1)) != 0;
                if (active && mine) {
                    const int kn = min(C, P - k0);
                    evals += (int64_t)nw * kn;
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
                if (j + 1 < total) {
                    // chunk j + 1 goes to the other buffer, whose chunk j - 1 every wave
                    // finished before the previous barrier
                    stash(lds + ((j + 1) & 1) * kChunkDoubles);
                    if (j + 2 < total)
                        fetch((s0 + list[j + 2]) * C);
                }
                __syncthreads();
            }
        }

        scan_finish<W, C, CHUNK_ARGMIN>(bx, by, bz, ld, P, n_valid, f, nw, offsets, drift, lambda,
                                        counter, evals, best, kbest, dsq);
    }
};

// The same scan with every wave on its own: no LDS and no block barrier. A wave tests
// each chunk as it comes (against min(ub, its running minimum), which only tightens
// the bound) and loads the points of the chunks it needs straight from memory; waves
// of a block that need the same chunk share it through the caches. With BUF (each
// coordinate's rows, from the tile's first seed on, span less than 4 GiB) the loads
// are buffer loads whose per-lane offset is fixed and whose row offset is a scalar,
// so no per-point address arithmetic runs on the vector unit.
template <int W, int C, bool CHUNK_ARGMIN, bool BUF, int SUP = 1>
struct TileScanDirect {
    static constexpr int kLdsDoubles = 1;

    // Arguments as TileScan::run (pairs and lds are unused; no synchronisation).
    __device__ static void run(const double *__restrict__ bx, const double *__restrict__ by,
                               const double *__restrict__ bz, int64_t ld, int P, int n_valid,
                               bool, const double (&f)[W][8], int nw,
                               const int32_t *__restrict__ offsets,
                               const double *__restrict__ drift, double lambda,
                               const double *__restrict__ rho, int64_t ldr,
                               unsigned long long *counter, double *, double (&dsq)[W])
    {
        static_assert(C % kRadiusChunk == 0 && C / kRadiusChunk <= 2, "chunk of 16 or 32");
        const int lane = threadIdx.x & 63;
        const bool active = nw > 0;
        const bool seed = lane < n_valid;
        const int64_t col = seed ? lane : 0;  // lanes without a seed read lane 0's column
        double best[W], cmin[W];
        float ub[W], sub[W];
        int kbest[W];
        int64_t evals = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            best[w] = INFINITY;
            kbest[w] = 0;
            ub[w] = INFINITY;
        }
        // The frames sit in scalar registers; an FMA may read only one scalar pair, so
        // the two offsets get vector copies once, not one per point.
        double fo[W][2];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            asm("v_mov_b64 %0, %1" : "=v"(fo[w][0]) : "s"(f[w][3]));
            asm("v_mov_b64 %0, %1" : "=v"(fo[w][1]) : "s"(f[w][7]));
        }
        auto proj_q = [&](int w, double x, double y, double z) {
            const double xi = fma(f[w][0], x, fma(f[w][1], y, fma(f[w][2], z, fo[w][0])));
            const double eta = fma(f[w][4], x, fma(f[w][5], y, fma(f[w][6], z, fo[w][1])));
            return fma(xi, xi, eta * eta);
        };
        const uint32_t voff = (uint32_t)col * 8u;
        // a raw buffer over one coordinate's rows (stride 0, no range limit); the base is
        // the same for the whole wave, and readfirstlane tells the compiler so
        auto rsrc = [](const double *p) {
            const uint64_t a = (uint64_t)p;
            const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(a >> 32))
                                << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
            return __builtin_amdgcn_make_buffer_rsrc((void *)u, 0, -1, 0x00020000);
        };
        auto load = [&](int k, double &x, double &y, double &z) {
            if constexpr (BUF) {
                const uint32_t soff = (uint32_t)k * (uint32_t)ld * 8u;  // wave-uniform
                x = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bx), voff, soff, 0));
                y = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(by), voff, soff, 0));
                z = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bz), voff, soff, 0));
            } else {
                const int64_t o = (int64_t)k * ld + col;
                x = bx[o];
                y = by[o];
                z = bz[o];
            }
        };
        if (active) {
            // (A) upper bounds of the final minima: every other chunk's first point
            int n_s = 0;
            for (int k0 = 0; k0 < P; k0 += 4 * C) {
                double x0, y0, z0, x1 = 0.0, y1 = 0.0, z1 = 0.0;
                load(k0, x0, y0, z0);
                const bool two = k0 + 2 * C < P;
                if (two)
                    load(k0 + 2 * C, x1, y1, z1);
                n_s += two ? 2 : 1;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    double xi, eta;
                    project(f[w], x0, y0, z0, xi, eta);
                    ub[w] = fminf(ub[w], (float)fma(xi, xi, eta * eta));
                    if (two) {
                        project(f[w], x1, y1, z1, xi, eta);
                        ub[w] = fminf(ub[w], (float)fma(xi, xi, eta * eta));
                    }
                }
            }
            evals += (int64_t)nw * n_s;
#pragma unroll
            for (int w = 0; w < W; ++w)
                sub[w] = __builtin_amdgcn_sqrtf(ub[w]) * 1.000001f;

            // Runs of SUP chunks first get one test from their first point with the sum
            // of their windows' radii (consecutive windows share their end points, so
            // every point of the run lies within that sum of its first point); a run
            // that no lane and wire needs is skipped whole, otherwise each chunk is
            // tested as usual. A run reaching past the track's end is tested per chunk.
            for (int s0 = 0; s0 < P; s0 += SUP * C) {
                const int s1 = min(P, s0 + SUP * C);
                if (SUP > 1 && s0 + SUP * C <= P) {
                    double x, y, z;
                    load(s0, x, y, z);
                    const int nr = s0 / kRadiusChunk;
                    double r = 0.0;
#pragma unroll
                    for (int i = 0; i < SUP * C / kRadiusChunk; ++i)
                        r = r + rho[(int64_t)(nr + i) * ldr + col];
                    const float rf = (float)r * 1.000001f;
                    bool lane_need = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const double q = proj_q(w, x, y, z);
                        if (w < nw) {
                            const float B = fmaf(rf + sub[w], 1.000001f, 1e-6f);
                            lane_need = lane_need ||
                                        !((float)q * 0.999999f > (B * B) * 1.000001f);
                        }
                    }
                    evals += nw;
                    if (__builtin_amdgcn_ballot_w64(lane_need && seed) == 0)
                        continue;
                }
                for (int k0 = s0; k0 < s1; k0 += C) {
                    const int kn = min(C, P - k0);
                    double x, y, z, q0[W];
                    load(k0, x, y, z);
                    double r = 0.0;
                    if (kn == C) {
                        const int nr = k0 / kRadiusChunk;
                        r = rho[(int64_t)nr * ldr + col];
                        if (C == 2 * kRadiusChunk)
                            r = r + rho[(int64_t)(nr + 1) * ldr + col];
                    }
                    const float rf = (float)r * 1.000001f;
                    bool lane_need = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        q0[w] = proj_q(w, x, y, z);
                        if (w < nw) {
                            const float B = fmaf(rf + sub[w], 1.000001f, 1e-6f);
                            lane_need = lane_need ||
                                        !((float)q0[w] * 0.999999f > (B * B) * 1.000001f);
                        }
                    }
                    evals += nw;
                    // the partial last chunk is always scanned
                    if (kn < C || __builtin_amdgcn_ballot_w64(lane_need && seed) != 0) {
                        evals += (int64_t)nw * (kn - 1);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            if (CHUNK_ARGMIN) {
                                cmin[w] = q0[w];
                            } else {
                                kbest[w] = q0[w] < best[w] ? k0 : kbest[w];
                                best[w] = fmin(best[w], q0[w]);
                            }
                        }
                        auto use = [&](int k, double px, double py, double pz) {
#pragma unroll
                            for (int w = 0; w < W; ++w) {
                                const double q = proj_q(w, px, py, pz);
                                if (CHUNK_ARGMIN) {
                                    cmin[w] = fmin(cmin[w], q);
                                } else {
                                    kbest[w] = q < best[w] ? k : kbest[w];
                                    best[w] = fmin(best[w], q);
                                }
                            }
                        };
                        if (kn == C) {
                            // points 1 .. C-1 in batches of 3, the next batch loading while
                            // the current one is used
                            constexpr int NB = (C + 1) / 3;
                            double cx[3], cy[3], cz[3];
                            auto load3 = [&](int b, double (&x)[3], double (&y)[3], double (&z)[3]) {
#pragma unroll
                                for (int i = 0; i < 3; ++i)
                                    if (1 + 3 * b + i < C)
                                        load(k0 + 1 + 3 * b + i, x[i], y[i], z[i]);
                            };
                            load3(0, cx, cy, cz);
#pragma unroll
                            for (int b = 0; b < NB; ++b) {
                                double nx[3], ny[3], nz[3];
                                if (b + 1 < NB)
                                    load3(b + 1, nx, ny, nz);
#pragma unroll
                                for (int i = 0; i < 3; ++i)
                                    if (1 + 3 * b + i < C)
                                        use(k0 + 1 + 3 * b + i, cx[i], cy[i], cz[i]);
#pragma unroll
                                for (int i = 0; i < 3; ++i) {
                                    cx[i] = nx[i];
                                    cy[i] = ny[i];
                                    cz[i] = nz[i];
                                }
                            }
                        } else {
                            for (int kk = 1; kk < kn; ++kk) {
                                double px, py, pz;
                                load(k0 + kk, px, py, pz);
                                use(k0 + kk, px, py, pz);
                            }
                        }
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            if (CHUNK_ARGMIN && cmin[w] < best[w]) {
                                best[w] = cmin[w];
                                kbest[w] = k0;
                            }
                            // the running minimum bounds the final one as well
                            sub[w] = fminf(sub[w],
                                           __builtin_amdgcn_sqrtf((float)best[w]) * 1.000001f);
                        }
                    }
                }
            }
        }
        scan_finish<W, C, CHUNK_ARGMIN>(bx, by, bz, ld, P, n_valid, f, nw, offsets, drift, lambda,
                                        counter, evals, best, kbest, dsq);
    }
};

// The wide form: one wave scans up to 16 wires, so that every chunk it reads serves
// many wires. The wires come in an order that keeps each wave's wires close in space
// (by azimuth), so they need nearly the same chunks. The frames sit in LDS (the
// block's wires, loaded once) and are read at each use, which leaves the vector
// registers to the chunk's points and the per-wire minima. Within a chunk that some
// wire needs, each wire is scanned only when some lane needs it for that wire (the
// same bound per wire), and its minimum is tracked per half chunk (the first index is
// recovered in the half that first reaches the final minimum, as in scan_finish). The
// next chunk's first point is loaded while the current chunk is scanned.
// CAP: the bound also uses the residual cap of Eq. 1. A wire's d is lambda whenever
// its DCA D exceeds its largest drift distance r_max plus lambda, so D is needed
// exactly only if some recorded point lies within cap = r_max + lambda + sigma (+ a
// margin) of the wire, sigma being the track's longest step. Every bound is then
// min(cap, the running minimum): if some point lies within the cap, the chunks holding
// the first minimum are never skipped and D is exact; if none does, every chord lies
// farther than r_max + lambda (a chord is within half its length, at most sigma / 2,
// of one of its end points), so whatever the scan finds gives d = lambda, exactly as
// the full scan. A wire without hits (d = lambda always) gets the cap 0. With the cap
// the pass over every other chunk's first point is not needed and is left out.
// EXACT: each evaluated point is compared with the running minimum, so the scan ends
// with the first index of the minimum itself (the definition: the first k whose q is
// below every earlier q) and the end needs only the three points of the chord
// refinement, not a rescan of the half chunk that holds it; each lane's rescan reads
// rows of its own, so the rescan costs far more HBM traffic than its point count says.
__device__ __forceinline__ float wide_cap(double rmax, double lambda, double sigma)
{
    if (rmax < 0.0)
        return 0.0f;
    return (float)((rmax + lambda) + sigma) * 1.000001f + 1e-5f;
}

template <int W, int SUP, bool BUF, bool CAP = false, bool EXACT = false, int HS = 0>
struct TileScanWide {
    static constexpr int C = kRadiusChunk;  // one radius window per chunk
    static constexpr int H = C / 2;         // the minimum is tracked per half chunk

    __device__ __forceinline__ static void frame(const double *fl, int w, double (&f)[8])
    {
        const double2 *p = reinterpret_cast<const double2 *>(fl + 8 * w);
        const double2 a = p[0], b = p[1], c = p[2], d = p[3];
        f[0] = a.x;
        f[1] = a.y;
        f[2] = b.x;
        f[3] = b.y;
        f[4] = c.x;
        f[5] = c.y;
        f[6] = d.x;
        f[7] = d.y;
    }
    __device__ __forceinline__ static double qf(const double (&f)[8], double x, double y, double z)
    {
        double xi, eta;
        project(f, x, y, z, xi, eta);
        return fma(xi, xi, eta * eta);
    }
    // the bound test of one (lane, wire): can a point within r of the tested point reach
    // or tie the wire's final minimum (bounded by sub)? Margins as in TileScanDirect.
    __device__ __forceinline__ static bool needs(double q0, float rf, float sub)
    {
        const float B = fmaf(rf + sub, 1.000001f, 1e-6f);
        return !((float)q0 * 0.999999f > (B * B) * 1.000001f);
    }

    // The end of a wide scan for one seed lane: per wire the first index of the minimum
    // within the SPAN points from kbest (eight loads at a time, no dependent load
    // chain), its chord refinement, D and Eq. 1's capped residual. With the cap, a wire
    // whose minimum stayed above the cap (or that no point came near) has every point
    // farther than r_max + lambda + the longest step, hence every chord farther than
    // r_max + lambda: its term is lambda^2, the full scan's, without a rescan.
    // EXACT_K: kbest already holds the first index (no rescan), and the three points of
    // four wires at a time are loaded before any of them is refined.
    template <int SPAN, bool CAPPED, bool EXACT_K = false>
    __device__ __forceinline__ static void finish(
        const double *__restrict__ bx, const double *__restrict__ by,
        const double *__restrict__ bz, int64_t ld, int P, int lane, const double *fl, int nw,
        const int32_t *__restrict__ wire_of, const int32_t *__restrict__ offsets,
        const double *__restrict__ drift, double lambda, const double (&best)[W],
        const int (&kbest)[W], const double *__restrict__ rmax, double sig, double (&dsq)[W])
    {
        if constexpr (EXACT_K) {
            // the three points of G wires are loaded before any of them is refined (one
            // round of loads per G wires instead of one per wire)
            constexpr int G = 4;
#pragma unroll
            for (int w0 = 0; w0 < W; w0 += G) {
                double pm[G][3], pc[G][3], pn[G][3];
                bool in[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int w = w0 + j;
                    in[j] = w < W && w < nw;
                    if constexpr (CAPPED) {
                        if (in[j]) {
                            const double c = (double)wide_cap(rmax[w], lambda, sig);
                            in[j] = best[w] <= c * c;
                        }
                    }
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        pm[j][a] = pc[j][a] = pn[j][a] = 0.0;
                    if (in[j]) {
                        const int k = kbest[w];
                        const int64_t o = (int64_t)k * ld + lane;
                        pc[j][0] = bx[o];
                        pc[j][1] = by[o];
                        pc[j][2] = bz[o];
                        if (k > 0) {
                            pm[j][0] = bx[o - ld];
                            pm[j][1] = by[o - ld];
                            pm[j][2] = bz[o - ld];
                        }
                        if (k < P - 1) {
                            pn[j][0] = bx[o + ld];
                            pn[j][1] = by[o + ld];
                            pn[j][2] = bz[o + ld];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int w = w0 + j;
                    if (w >= W || w >= nw)
                        continue;
                    if (!in[j]) {
                        // CAPPED: every chord farther than r_max + lambda
                        dsq[w] = lambda * lambda;
                        continue;
                    }
                    double f[8];
                    frame(fl, w, f);
                    const double d2 = refine_dca2_at(f, kbest[w], P, best[w], pm[j], pc[j], pn[j]);
                    const double D = sqrt(d2);
                    const int wi = wire_of[w];
                    const double d = capped_residual(D, drift, offsets[wi], offsets[wi + 1], lambda);
                    dsq[w] = d * d;
                }
            }
            return;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (w >= nw)
                continue;
            if constexpr (CAPPED) {
                const double c = (double)wide_cap(rmax[w], lambda, sig);
                if (!(best[w] <= c * c)) {
                    dsq[w] = lambda * lambda;
                    continue;
                }
            }
            double f[8];
            frame(fl, w, f);
            const int k = kbest[w];
            int kf = k;
            if constexpr (!EXACT_K) {
                kf = -1;
                for (int h0 = 0; h0 < SPAN && kf < 0; h0 += 8) {
                    double q[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int j = k + h0 + i;
                        q[i] = NAN;  // never equal: past the track's end
                        if (j < P) {
                            const int64_t o = (int64_t)j * ld + lane;
                            q[i] = qf(f, bx[o], by[o], bz[o]);
                        }
                    }
#pragma unroll
                    for (int i = 7; i >= 0; --i)
                        if (q[i] == best[w])
                            kf = k + h0 + i;
                }
                if (kf < 0)
                    kf = k;
            }
            const double d2 = refine_dca2(bx + lane, by + lane, bz + lane, ld, P, f, kf, best[w]);
            const double D = sqrt(d2);
            const int wi = wire_of[w];
            const double d = capped_residual(D, drift, offsets[wi], offsets[wi + 1], lambda);
            dsq[w] = d * d;
        }
    }

    // bx, by, bz: the tile's track (point k of lane l at b[k * ld + l]); fl: this wave's
    // W frames in LDS ([W][8], slots >= nw hold anything finite); wire_of: the wave's
    // slots' wire indices (CSR rows of offsets/drift); rho: the tile's chunk radii, with
    // each track's longest step in row radius_chunks(P); rmax (CAP): the wave's slots'
    // largest drift distances (-1: no hits).
    // Returns d^2 of (lane, slot w) in dsq[w] for lanes < n_valid and w < nw.
    __device__ __forceinline__ static void run(
        const double *__restrict__ bx, const double *__restrict__ by,
        const double *__restrict__ bz, int64_t ld, int P, int n_valid, const double *fl, int nw,
        const int32_t *__restrict__ wire_of, const int32_t *__restrict__ offsets,
        const double *__restrict__ drift, double lambda, const double *__restrict__ rho,
        int64_t ldr, unsigned long long *counter, double (&dsq)[W],
        const double *__restrict__ rmax = nullptr)
    {
        const int lane = threadIdx.x & 63;
        const bool seed = lane < n_valid;
        const int64_t col = seed ? lane : 0;  // lanes without a seed read lane 0's column
        double best[W];
        float sub[W];
        int kbest[W];
        int64_t evals = 0;  // wave-uniform, per seed lane
#pragma unroll
        for (int w = 0; w < W; ++w) {
            best[w] = INFINITY;
            kbest[w] = 0;
            sub[w] = INFINITY;
        }
        const uint32_t voff = (uint32_t)col * 8u;
        auto rsrc = [](const double *p) {
            const uint64_t a = (uint64_t)p;
            const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(a >> 32))
                                << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
            return __builtin_amdgcn_make_buffer_rsrc((void *)u, 0, -1, 0x00020000);
        };
        auto load = [&](int k, double &x, double &y, double &z) {
            if constexpr (BUF) {
                const uint32_t soff = (uint32_t)k * (uint32_t)ld * 8u;  // wave-uniform
                x = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bx), voff, soff, 0));
                y = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(by), voff, soff, 0));
                z = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bz), voff, soff, 0));
            } else {
                const int64_t o = (int64_t)k * ld + col;
                x = bx[o];
                y = by[o];
                z = bz[o];
            }
        };
        double sig = 0.0;  // the track's longest step (the cap)
        if (CAP && nw > 0) {
            sig = rho[(int64_t)radius_chunks(P) * ldr + col];
#pragma unroll
            for (int w = 0; w < W; ++w)
                sub[w] = w < nw ? wide_cap(rmax[w], lambda, sig) : 0.0f;
        }
        if constexpr (EXACT && HS > 0 && CAP) {
            // Chunk parts (HS > 0). Every test measures from the middle of its stretch, all
            // of whose points lie within half its length times sig (the track's longest
            // step) of that point: a run of SUP chunks from its point SUP C / 2, a chunk
            // from its point C / 2, and each of the HS parts of a needed chunk, per wire,
            // from its own middle point; a part is scanned only where some lane's bound
            // needs it. The next chunk's middle point loads while the current chunk is
            // tested and scanned.
            constexpr int L = C / HS;  // points per part
            static_assert(L * HS == C && L > 1, "parts of a chunk");
            const float r_run = (float)(sig * (SUP * C / 2)) * 1.000001f;
            const float r_chk = (float)(sig * (C / 2)) * 1.000001f;
            const float r_prt = (float)(sig * (L / 2)) * 1.000001f;
            const int nch = (P + C - 1) / C;
            double mx = 0.0, my = 0.0, mz = 0.0;  // chunk n's middle point, when m_ok
            bool m_ok = false;
            for (int n = 0; nw > 0 && n < nch;) {
                __asm__ volatile("" ::: "memory");  // frames are re-read from LDS below
                const int k0 = n * C;
                const int kn = min(C, P - k0);
                if (SUP > 1 && n % SUP == 0 && k0 + SUP * C <= P) {
                    double rx, ry, rz;
                    load(k0 + SUP * C / 2, rx, ry, rz);
                    if (!m_ok) {
                        load(k0 + C / 2, mx, my, mz);
                        m_ok = true;
                    }
                    bool lane_need = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        frame(fl, w, f);
                        lane_need = lane_need || (w < nw && needs(qf(f, rx, ry, rz), r_run, sub[w]));
                    }
                    evals += nw;
                    if (__builtin_amdgcn_ballot_w64(lane_need && seed) == 0) {
                        n += SUP;
                        m_ok = false;
                        continue;
                    }
                }
                if (kn == C) {
                    if (!m_ok)
                        load(k0 + C / 2, mx, my, mz);
                    const bool next_full = (n + 2) * C <= P;
                    double nx = 0.0, ny = 0.0, nz = 0.0;
                    if (next_full)
                        load(k0 + C + C / 2, nx, ny, nz);
                    uint32_t needm = 0;  // wave-uniform: the wires some lane needs here
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        frame(fl, w, f);
                        const bool ln = w < nw && needs(qf(f, mx, my, mz), r_chk, sub[w]);
                        if (__builtin_amdgcn_ballot_w64(ln && seed) != 0)
                            needm |= 1u << w;
                    }
                    evals += nw;
                    if (needm != 0) {
                        double x[C], y[C], z[C];
#pragma unroll
                        for (int i = 0; i < C; ++i)
                            load(k0 + i, x[i], y[i], z[i]);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            if ((needm >> w) & 1u) {
                                double f[8];
                                frame(fl, w, f);
                                double b = best[w];
                                int kb = kbest[w];
#pragma unroll
                                for (int g = 0; g < HS; ++g) {
                                    const int i0 = g * L, im = i0 + L / 2;
                                    const double qm = qf(f, x[im], y[im], z[im]);
                                    if (__builtin_amdgcn_ballot_w64(needs(qm, r_prt, sub[w]) && seed) != 0) {
                                        // point by point, in order (the middle one's q reused)
#pragma unroll
                                        for (int i = i0; i < i0 + L; ++i) {
                                            const double q = i == im ? qm : qf(f, x[i], y[i], z[i]);
                                            kb = q < b ? k0 + i : kb;
                                            b = fmin(b, q);
                                        }
                                        evals += L - 1;
                                    }
                                }
                                evals += HS;  // the parts' middle points
                                best[w] = b;
                                kbest[w] = kb;
                                // the running minimum bounds the final one as well
                                sub[w] = fminf(sub[w], __builtin_amdgcn_sqrtf((float)b) * 1.000001f);
                            }
                        }
                    }
                    mx = nx;
                    my = ny;
                    mz = nz;
                    m_ok = next_full;
                } else {
                    // the partial last chunk: every wire, every point
                    double x[C], y[C], z[C];
#pragma unroll
                    for (int i = 0; i < C; ++i) {
                        x[i] = y[i] = z[i] = 0.0;
                        if (i < kn)
                            load(k0 + i, x[i], y[i], z[i]);
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        if (w < nw) {
                            double f[8];
                            frame(fl, w, f);
                            double b = best[w];
                            int kb = kbest[w];
#pragma unroll
                            for (int i = 0; i < C; ++i) {
                                if (i < kn) {
                                    const double q = qf(f, x[i], y[i], z[i]);
                                    kb = q < b ? k0 + i : kb;
                                    b = fmin(b, q);
                                }
                            }
                            best[w] = b;
                            kbest[w] = kb;
                        }
                    }
                    evals += (int64_t)nw * kn;
                    m_ok = false;
                }
                ++n;
            }
        }
        if (!(EXACT && HS > 0 && CAP) && nw > 0) {
            // (A) upper bounds of the final minima: every other chunk's first point, eight
            // points per pass, each frame read once per pass (not needed with the cap)
            float ub[W];
#pragma unroll
            for (int w = 0; w < W; ++w)
                ub[w] = INFINITY;
            int n_s = 0;
            for (int k0 = 0; !CAP && k0 < P; k0 += 8 * 2 * C) {
                double x[8], y[8], z[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    x[i] = y[i] = z[i] = 0.0;
                    if (k0 + i * 2 * C < P)
                        load(k0 + i * 2 * C, x[i], y[i], z[i]);
                }
                n_s += min(8, (P - 1 - k0) / (2 * C) + 1);
                __asm__ volatile("" ::: "memory");
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    double f[8];
                    frame(fl, w, f);
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (k0 + i * 2 * C < P)
                            ub[w] = fminf(ub[w], (float)qf(f, x[i], y[i], z[i]));
                }
            }
            evals += (int64_t)nw * n_s;
            if (!CAP)
#pragma unroll
                for (int w = 0; w < W; ++w)
                    sub[w] = __builtin_amdgcn_sqrtf(ub[w]) * 1.000001f;

            const int nch = (P + C - 1) / C;
            double cx, cy, cz;  // the first point of chunk n
            load(0, cx, cy, cz);
            for (int n = 0; n < nch;) {
                __asm__ volatile("" ::: "memory");  // frames are re-read from LDS below
                const int k0 = n * C;
                if (SUP > 1 && n % SUP == 0 && k0 + SUP * C <= P) {
                    // a run of SUP chunks: one test with the sum of its windows' radii
                    double r = 0.0;
#pragma unroll
                    for (int i = 0; i < SUP; ++i)
                        r = r + rho[(int64_t)(n + i) * ldr + col];
                    const float rf = (float)r * 1.000001f;
                    bool lane_need = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        frame(fl, w, f);
                        lane_need = lane_need || (w < nw && needs(qf(f, cx, cy, cz), rf, sub[w]));
                    }
                    evals += nw;
                    if (__builtin_amdgcn_ballot_w64(lane_need && seed) == 0) {
                        n += SUP;
                        if (n < nch)
                            load(n * C, cx, cy, cz);
                        continue;
                    }
                }
                const int kn = min(C, P - k0);
                double nx = 0.0, ny = 0.0, nz = 0.0;
                if (n + 1 < nch)
                    load(k0 + C, nx, ny, nz);
                if (kn == C) {
                    const float rf = (float)rho[(int64_t)n * ldr + col] * 1.000001f;
                    uint32_t needm = 0;  // wave-uniform: the wires some lane needs here
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        frame(fl, w, f);
                        const bool ln = w < nw && needs(qf(f, cx, cy, cz), rf, sub[w]);
                        if (__builtin_amdgcn_ballot_w64(ln && seed) != 0)
                            needm |= 1u << w;
                    }
                    evals += nw;
                    if (needm != 0) {
                        double x[C - 1], y[C - 1], z[C - 1];
#pragma unroll
                        for (int i = 1; i < C; ++i)
                            load(k0 + i, x[i - 1], y[i - 1], z[i - 1]);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            if ((needm >> w) & 1u) {
                                double f[8];
                                frame(fl, w, f);
                                if constexpr (EXACT) {
                                    // point by point: k replaces kbest only below the
                                    // running minimum (fmin equals that select here: the
                                    // minimum is never NaN and q is never -0)
                                    double b = best[w];
                                    int kb = kbest[w];
                                    double q = qf(f, cx, cy, cz);
                                    kb = q < b ? k0 : kb;
                                    b = fmin(b, q);
#pragma unroll
                                    for (int i = 1; i < C; ++i) {
                                        q = qf(f, x[i - 1], y[i - 1], z[i - 1]);
                                        kb = q < b ? k0 + i : kb;
                                        b = fmin(b, q);
                                    }
                                    best[w] = b;
                                    kbest[w] = kb;
                                } else {
                                    double m = qf(f, cx, cy, cz);
#pragma unroll
                                    for (int i = 1; i < H; ++i)
                                        m = fmin(m, qf(f, x[i - 1], y[i - 1], z[i - 1]));
                                    if (m < best[w]) {
                                        best[w] = m;
                                        kbest[w] = k0;
                                    }
                                    m = qf(f, x[H - 1], y[H - 1], z[H - 1]);
#pragma unroll
                                    for (int i = H + 1; i < C; ++i)
                                        m = fmin(m, qf(f, x[i - 1], y[i - 1], z[i - 1]));
                                    if (m < best[w]) {
                                        best[w] = m;
                                        kbest[w] = k0 + H;
                                    }
                                }
                                // the running minimum bounds the final one as well
                                sub[w] = fminf(sub[w],
                                               __builtin_amdgcn_sqrtf((float)best[w]) * 1.000001f);
                                evals += C - 1;
                            }
                        }
                    }
                } else {
                    // the partial last chunk: every wire, every point
                    double x[C - 1], y[C - 1], z[C - 1];
#pragma unroll
                    for (int i = 1; i < C; ++i) {
                        x[i - 1] = y[i - 1] = z[i - 1] = 0.0;
                        if (i < kn)
                            load(k0 + i, x[i - 1], y[i - 1], z[i - 1]);
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        if (w < nw) {
                            double f[8];
                            frame(fl, w, f);
                            if constexpr (EXACT) {
                                double b = best[w];
                                int kb = kbest[w];
                                double q = qf(f, cx, cy, cz);
                                kb = q < b ? k0 : kb;
                                b = fmin(b, q);
#pragma unroll
                                for (int i = 1; i < C; ++i) {
                                    if (i < kn) {
                                        q = qf(f, x[i - 1], y[i - 1], z[i - 1]);
                                        kb = q < b ? k0 + i : kb;
                                        b = fmin(b, q);
                                    }
                                }
                                best[w] = b;
                                kbest[w] = kb;
                            } else {
                                double m = qf(f, cx, cy, cz);
#pragma unroll
                                for (int i = 1; i < C; ++i)
                                    if (i < kn)
                                        m = fmin(m, qf(f, x[i - 1], y[i - 1], z[i - 1]));
                                if (m < best[w]) {
                                    best[w] = m;
                                    kbest[w] = k0;
                                }
                            }
                        }
                    }
                    evals += (int64_t)nw * kn;
                }
                cx = nx;
                cy = ny;
                cz = nz;
                ++n;
            }
        }
        // the end: evaluation count, then per (lane, wire) the first index of the
        // minimum (EXACT: already known; else a rescan of the half chunk that holds it),
        // its chord refinement, D and Eq. 1's capped residual
        if (counter && lane == 0 && evals > 0)
            atomicAdd(counter, (unsigned long long)(evals * n_valid));
#pragma unroll
        for (int w = 0; w < W; ++w)
            dsq[w] = 0.0;
        if (nw <= 0 || !seed)
            return;
        // the last chunk may hold up to C points in its one recorded span
        finish<C, CAP, EXACT>(bx, by, bz, ld, P, lane, fl, nw, wire_of, offsets, drift, lambda,
                              best, kbest, rmax, sig, dsq);
    }
};

// The wide form with its memory latency hidden. The chunks are taken NB at a time: the
// first points of all NB come in one round of loads, and every (chunk, wire) of the
// batch is tested against the bounds as they stand before the batch (a bound only
// tightens, so an older one is still valid); a batch whose first point, with the sum
// of its windows' radii, rules out every lane and wire is passed over. The chunks the
// batch needs are then scanned in half chunks of H points with two register buffers:
// the next half is loading while the current one is evaluated. Each wire of a chunk
// is evaluated only where some lane needs it; its minimum is tracked per half chunk.
template <int W, int NB, bool BUF, bool CAP = false>
struct TileScanWideP {
    using Base = TileScanWide<W, 1, BUF>;
    static constexpr int C = kRadiusChunk;
    static constexpr int H = C / 2;

    __device__ __forceinline__ static void run(
        const double *__restrict__ bx, const double *__restrict__ by,
        const double *__restrict__ bz, int64_t ld, int P, int n_valid, const double *fl, int nw,
        const int32_t *__restrict__ wire_of, const int32_t *__restrict__ offsets,
        const double *__restrict__ drift, double lambda, const double *__restrict__ rho,
        int64_t ldr, unsigned long long *counter, double (&dsq)[W],
        const double *__restrict__ rmax = nullptr)
    {
        const int lane = threadIdx.x & 63;
        const bool seed = lane < n_valid;
        const int64_t col = seed ? lane : 0;  // lanes without a seed read lane 0's column
        double best[W];
        float sub[W];
        int kbest[W];
        int64_t evals = 0;  // wave-uniform, per seed lane
#pragma unroll
        for (int w = 0; w < W; ++w) {
            best[w] = INFINITY;
            kbest[w] = 0;
            sub[w] = INFINITY;
        }
        const uint32_t voff = (uint32_t)col * 8u;
        auto rsrc = [](const double *p) {
            const uint64_t a = (uint64_t)p;
            const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(a >> 32))
                                << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
            return __builtin_amdgcn_make_buffer_rsrc((void *)u, 0, -1, 0x00020000);
        };
        auto load = [&](int k, double &x, double &y, double &z) {
            if constexpr (BUF) {
                const uint32_t soff = (uint32_t)k * (uint32_t)ld * 8u;  // wave-uniform
                x = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bx), voff, soff, 0));
                y = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(by), voff, soff, 0));
                z = __builtin_bit_cast(double,
                                       __builtin_amdgcn_raw_buffer_load_b64(rsrc(bz), voff, soff, 0));
            } else {
                const int64_t o = (int64_t)k * ld + col;
                x = bx[o];
                y = by[o];
                z = bz[o];
            }
        };
        // points k0 .. k0 + H - 1 (those below P; 0 elsewhere)
        auto load_half = [&](int k0, double (&x)[H], double (&y)[H], double (&z)[H]) {
#pragma unroll
            for (int i = 0; i < H; ++i) {
                x[i] = y[i] = z[i] = 0.0;
                if (k0 + i < P)
                    load(k0 + i, x[i], y[i], z[i]);
            }
        };
        // the first n points (n wave-uniform, 1..H) of a half starting at k0, for the
        // wires in mask: per wire the half's minimum, recorded when it beats the best
        // The compiler fences keep each frame's LDS read next to its use (no frame is
        // hoisted out of the loops), so at most two frames are live: the next wire's
        // frame loads while the current one is evaluated.
        auto eval_half = [&](int k0, int n, uint32_t mask, const double (&x)[H],
                             const double (&y)[H], const double (&z)[H]) {
            double f[8];
            Base::frame(fl, 0, f);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double fn[8];
                __asm__ volatile("" ::: "memory");
                if (w + 1 < W)
                    Base::frame(fl, w + 1, fn);
                if ((mask >> w) & 1u) {
                    double m = Base::qf(f, x[0], y[0], z[0]);
#pragma unroll
                    for (int i = 1; i < H; ++i)
                        if (i < n)  // wave-uniform; every point of a full half
                            m = fmin(m, Base::qf(f, x[i], y[i], z[i]));
                    if (m < best[w]) {
                        best[w] = m;
                        kbest[w] = k0;
                    }
                }
                if (w + 1 < W)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        f[j] = fn[j];
            }
            evals += (int64_t)__builtin_popcount(mask) * n;
        };
        double sig = 0.0;  // the track's longest step (the cap)
        if (CAP && nw > 0) {
            sig = rho[(int64_t)radius_chunks(P) * ldr + col];
#pragma unroll
            for (int w = 0; w < W; ++w)
                sub[w] = w < nw ? wide_cap(rmax[w], lambda, sig) : 0.0f;
        }
        if (nw > 0) {
            // (A) upper bounds of the final minima: every other chunk's first point,
            // eight per round, the next round loading while this one is evaluated (not
            // needed with the cap)
            float ub[W];
#pragma unroll
            for (int w = 0; w < W; ++w)
                ub[w] = INFINITY;
            int n_s = 0;
            if (!CAP) {
                double x[8], y[8], z[8];
                auto load8 = [&](int k0, double (&px)[8], double (&py)[8], double (&pz)[8]) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        px[i] = py[i] = pz[i] = 0.0;
                        if (k0 + i * 2 * C < P)
                            load(k0 + i * 2 * C, px[i], py[i], pz[i]);
                    }
                };
                load8(0, x, y, z);
                for (int k0 = 0; k0 < P; k0 += 8 * 2 * C) {
                    double nx[8], ny[8], nz[8];
                    if (k0 + 8 * 2 * C < P)
                        load8(k0 + 8 * 2 * C, nx, ny, nz);
                    n_s += min(8, (P - 1 - k0) / (2 * C) + 1);
                    __asm__ volatile("" ::: "memory");
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        __asm__ volatile("" ::: "memory");
                        Base::frame(fl, w, f);
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (k0 + i * 2 * C < P)
                                ub[w] = fminf(ub[w], (float)Base::qf(f, x[i], y[i], z[i]));
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        x[i] = nx[i];
                        y[i] = ny[i];
                        z[i] = nz[i];
                    }
                }
            }
            evals += (int64_t)nw * n_s;
            if (!CAP)
#pragma unroll
                for (int w = 0; w < W; ++w)
                    sub[w] = __builtin_amdgcn_sqrtf(ub[w]) * 1.000001f;
            const uint32_t all = nw >= 32 ? 0xffffffffu : ((1u << nw) - 1u);

            const int nch = (P + C - 1) / C;
            for (int b0 = 0; b0 < nch; b0 += NB) {
                __asm__ volatile("" ::: "memory");  // frames are re-read from LDS below
                const int nb = min(NB, nch - b0);
                uint32_t needm[NB];
                {
                    double px[NB], py[NB], pz[NB], r[NB];
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        px[i] = py[i] = pz[i] = r[i] = 0.0;
                        if (i < nb) {
                            load((b0 + i) * C, px[i], py[i], pz[i]);
                            if ((b0 + i) * C + C <= P)
                                r[i] = rho[(int64_t)(b0 + i) * ldr + col];
                        }
                    }
                    // the whole batch from its first point, with the sum of its windows'
                    // radii (consecutive windows share their end points)
                    bool any = true;
                    if (nb == NB && (b0 + NB) * C <= P) {
                        double rs = 0.0;
#pragma unroll
                        for (int i = 0; i < NB; ++i)
                            rs = rs + r[i];
                        const float rf = (float)rs * 1.000001f;
                        bool lane_need = false;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            double f[8];
                            Base::frame(fl, w, f);
                            lane_need = lane_need ||
                                        (w < nw && Base::needs(Base::qf(f, px[0], py[0], pz[0]),
                                                               rf, sub[w]));
                        }
                        evals += nw;
                        any = __builtin_amdgcn_ballot_w64(lane_need && seed) != 0;
                    }
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        needm[i] = 0;
                    if (!any)
                        continue;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double f[8];
                        __asm__ volatile("" ::: "memory");
                        Base::frame(fl, w, f);
#pragma unroll
                        for (int i = 0; i < NB; ++i) {
                            if (i < nb) {
                                const float rf = (float)r[i] * 1.000001f;
                                const bool ln = w < nw && Base::needs(
                                                              Base::qf(f, px[i], py[i], pz[i]),
                                                              rf, sub[w]);
                                if (__builtin_amdgcn_ballot_w64(ln && seed) != 0)
                                    needm[i] |= 1u << w;
                            }
                        }
                    }
                    evals += (int64_t)nw * nb;
                    // the partial last chunk is always scanned, every wire
                    if ((b0 + nb) * C > P)
                        needm[nb - 1] = all;
                }
                uint32_t act = 0;  // the batch's chunks some wire needs
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    act |= (needm[i] != 0 ? 1u : 0u) << i;
                if (act == 0)
                    continue;
                double ax[H], ay[H], az[H], cx[H], cy[H], cz[H];
                int i = __builtin_ctz(act);
                load_half((b0 + i) * C, ax, ay, az);
                while (true) {
                    __asm__ volatile("" ::: "memory");
                    const int k0 = (b0 + i) * C;
                    const int kn = min(C, P - k0);
                    uint32_t m = 0;
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        m = j == i ? needm[j] : m;
                    if (kn > H)
                        load_half(k0 + H, cx, cy, cz);
                    eval_half(k0, min(H, kn), m, ax, ay, az);
                    const uint32_t rest = act & ~((2u << i) - 1u);
                    const int nxt = rest ? __builtin_ctz(rest) : -1;
                    if (nxt >= 0)
                        load_half((b0 + nxt) * C, ax, ay, az);
                    if (kn > H)
                        eval_half(k0 + H, kn - H, m, cx, cy, cz);
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        if ((m >> w) & 1u)
                            sub[w] = fminf(sub[w],
                                           __builtin_amdgcn_sqrtf((float)best[w]) * 1.000001f);
                    if (nxt < 0)
                        break;
                    i = nxt;
                }
            }
        }
        // the end, as TileScanWide: the first index of the minimum within its half chunk,
        // its chord refinement, D and Eq. 1's capped residual
        if (counter && lane == 0 && evals > 0)
            atomicAdd(counter, (unsigned long long)(evals * n_valid));
#pragma unroll
        for (int w = 0; w < W; ++w)
            dsq[w] = 0.0;
        if (nw <= 0 || !seed)
            return;
        Base::template finish<H, CAP>(bx, by, bz, ld, P, lane, fl, nw, wire_of, offsets, drift,
                                      lambda, best, kbest, rmax, sig, dsq);
    }
};

}  // namespace cdev

#endif  // COMET_DCA_SCAN_H
