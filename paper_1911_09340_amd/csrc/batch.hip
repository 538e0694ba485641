// batch.hip -- the seed scan of many events with uneven hit and turn counts in
// persistent launches: every turn partition of every event goes through the paper's
// Sec. 2.1 path (grid scan, argmin, finer re-scans, classification).
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 2 (Alg. 1-3, Eq. 1).
//
// Events are packed in one CSR (event -> wires -> hits); partition p belongs to event
// part_event[p] and scans the grid descriptor grids[p] (the same n per axis for all
// partitions, S seeds). The scan kernel is persistent: each block takes work items
// (a partition and up to one tile of 64 seeds per wave) from an atomic work counter
// until none are left. Every wave builds its tile's seeds from the partition's
// descriptor and records their RK4 tracks into the block's own scratch rows; then the
// block scans the tiles one by one against the partition's event wires, group by
// group, with the same tile scan as the single-event kernel (cdev::TileScan). Each
// wire group's d^2 values go to LDS and one wave adds them to the per-seed RSS in
// wire order, so every RSS equals the single-event path's bit for bit.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "comet.h"
#include "dca_scan.h"
#include "device_math.h"
#include "field_math.h"
#include "host_common.h"

namespace {

using namespace cdev;
using namespace chost;

constexpr int kMaxBatchBlocks = 512;  // persistent blocks at most (2 per CU on gfx950)
constexpr int kMaxBatchNwv = 8;       // waves per block at most = tiles per work item
constexpr int kBatchWirePad = 64;     // frames padding: at least one wire group W * NWV

struct BatchArgs {
    const double *frames;     // [W_pad][8]
    const int32_t *offsets;   // [W + 1] global hit CSR
    const double *drift;      // [H]
    const int32_t *ev_wires;  // [E + 1]
    const int32_t *part_event;
    const double *grids;      // [NP][14]
    int n0, n1, n2, n3;
    int64_t S;
    int tiles;                // 64-seed tiles per partition
    int supers;               // work items (super-tiles of NWV tiles) per partition
    int64_t n_items;          // partitions x supers
    int64_t max_tiles;        // tiles (partition-major) scanned, at most partitions x tiles
    double bz, charge, h, lambda;
    int K;
    double *scratch;          // [blocks][NWV] x ([3][P][64] tracks, [P/16][64] chunk radii)
    int *counter;             // work queue
    int *done;                // [NP] tiles finished per partition
    double *rss;              // [NP][S]
    int64_t *best;            // [NP]
    unsigned long long *evals;  // profiling: distance evaluations, or null
    FieldMap fm;              // the field map of the FIELD kernel (tracks as field.hip records them)
    const int32_t *active;    // [E] or null: the partitions of events with active[e] == 0 are skipped
    // wires in azimuth order within each event (slot r holds wire wire_of_az[r], its frame
    // and its largest drift distance)
    const double *frames_az;
    const int32_t *wire_of_az;
    const double *caps_az;
};

// One seed's track in the map into a tile's scratch rows (stride 64) with its chunk
// radii: the steps of rk4_field_record_kernel (RK4, or RKN for fm.stepper 1).
__device__ __forceinline__ void record_field_track(const FieldMap &fm, const double (&st)[6],
                                                   double charge, double h, int K,
                                                   double *sx, double *sy, double *sz,
                                                   double *rho, int lane)
{
    const int P = K + 1;
    double x[3] = {st[0], st[1], st[2]}, p[3] = {st[3], st[4], st[5]};
    const double p0 = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const double inv = 1.0 / p0;
    const double g = (kKappa * charge) * inv;
    const bool rkn = fm.stepper == 1;
    const RknConsts kn = rkn_consts(h);
    if (rkn)
        for (int c = 0; c < 3; ++c)
            p[c] = p[c] * inv;
    ChunkRadius rad;
    for (int k = 0; k < K; ++k) {
        sx[(int64_t)k * 64 + lane] = x[0];
        sy[(int64_t)k * 64 + lane] = x[1];
        sz[(int64_t)k * 64 + lane] = x[2];
        if (rho)
            rad.add(k, P, x[0], x[1], x[2], rho, 64);
        if (rkn)
            rkn_field_step(fm, kn, g, x, p);
        else
            rk4_field_step(fm, inv, g, h, x, p);
    }
    sx[(int64_t)K * 64 + lane] = x[0];
    sy[(int64_t)K * 64 + lane] = x[1];
    sz[(int64_t)K * 64 + lane] = x[2];
    if (rho)
        rad.add(K, P, x[0], x[1], x[2], rho, 64);
}

// WPE: waves per SIMD the register allocation must allow (2 blocks of 8 waves per CU
// need 4). A work item is a super-tile of up to NWV consecutive 64-seed tiles of one
// partition: every wave records one tile's tracks (RK4 runs on all waves at once),
// then the block scans the tiles one after the other against the event's wires.
template <int W, int NWV, int C, int WPE, bool DIRECT, bool FIELD = false, int SUP = 1>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(WPE))) void
batch_scan_kernel(BatchArgs a)
{
    using Scan = std::conditional_t<DIRECT, TileScanDirect<W, C, true, true, SUP>,
                                    TileScan<W, NWV, C, true>>;
    constexpr int G = W * NWV;  // wires per group
    static_assert(NWV <= kMaxBatchNwv && G <= kBatchWirePad, "shape exceeds the workspace");
    __shared__ __align__(16) double lds[Scan::kLdsDoubles];
    __shared__ double dd[G * 64];
    __shared__ int item_s;
    __shared__ int last_s;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = a.K + 1;
    const int64_t row = (int64_t)P * 64;                 // one coordinate of one tile
    const int64_t rrow = (int64_t)radius_rows(P) * 64;  // chunk radii and longest step of one tile
    double *const block_scratch = a.scratch + (int64_t)blockIdx.x * NWV * (3 * row + rrow);
    double *const block_rho = block_scratch + (int64_t)NWV * 3 * row;

    // Control flow around the barriers stays wave-uniform: counters are bumped by a
    // whole wave (lane 0 adds its count, the others 0) and results are broadcast with
    // readfirstlane, never by a region that only thread 0 enters (the compiler may
    // move such a region across the loop's back edge, apart from its wave's barriers).
    for (;;) {
        if (wave == 0) {
            const int old = atomicAdd(a.counter, lane == 0 ? 1 : 0);
            item_s = __builtin_amdgcn_readfirstlane(old);
        }
        __syncthreads();
        const int64_t item = __builtin_amdgcn_readfirstlane(item_s);
        __syncthreads();
        if (item >= a.n_items)
            break;
        const int p = (int)(item / a.supers);
        const int t0 = (int)(item - (int64_t)p * a.supers) * NWV;  // first tile
        // tiles of this item that exist and lie within the max_tiles prefix
        const int64_t first_global = (int64_t)p * a.tiles + t0;
        const int n_sub = (int)max((int64_t)0, min(min((int64_t)NWV, (int64_t)(a.tiles - t0)),
                                                   a.max_tiles - first_global));
        const int e = a.part_event[p];
        if (a.active && a.active[e] == 0)
            continue;  // block-uniform: the whole item is skipped, the partition keeps best -1
        const int w0 = a.ev_wires[e], w1 = a.ev_wires[e + 1];

        // seeds and tracks: wave w records tile t0 + w (one seed per lane)
        if (wave < n_sub) {
            const int64_t s0 = (int64_t)(t0 + wave) * 64;
            const int n_valid = (int)min((int64_t)64, a.S - s0);
            double *sx = block_scratch + (int64_t)wave * 3 * row;
            double *sy = sx + row, *sz = sy + row;
            double *rho = block_rho + (int64_t)wave * rrow + lane;
            if constexpr (FIELD) {
                if (lane < n_valid) {
                    double st[6];
                    seed_from_grid(a.grids + 14 * (int64_t)p, a.n0, a.n1, a.n2, a.n3,
                                   s0 + lane, st);
                    record_field_track(a.fm, st, a.charge, a.h, a.K, sx, sy, sz, rho, lane);
                }
            } else if (lane < n_valid) {
                ChunkRadius rad;
                double st[6];
                seed_from_grid(a.grids + 14 * (int64_t)p, a.n0, a.n1, a.n2, a.n3, s0 + lane,
                               st);
                double x = st[0], y = st[1], z = st[2], px = st[3], py = st[4];
                const StepConsts kc = step_consts(px, py, st[5], a.bz, a.charge, a.h);
                for (int k = 0; k < a.K; ++k) {
                    sx[(int64_t)k * 64 + lane] = x;
                    sy[(int64_t)k * 64 + lane] = y;
                    sz[(int64_t)k * 64 + lane] = z;
                    rad.add(k, P, x, y, z, rho, 64);
                    rk4_step(kc, x, y, z, px, py);
                }
                sx[(int64_t)a.K * 64 + lane] = x;
                sy[(int64_t)a.K * 64 + lane] = y;
                sz[(int64_t)a.K * 64 + lane] = z;
                rad.add(a.K, P, x, y, z, rho, 64);
            }
        }
        __syncthreads();

        for (int t = 0; t < n_sub; ++t) {
            const int64_t s0 = (int64_t)(t0 + t) * 64;
            const int n_valid = (int)min((int64_t)64, a.S - s0);
            const double *sx = block_scratch + (int64_t)t * 3 * row;
            const double *sy = sx + row, *sz = sy + row;
            double acc = 0.0;  // RSS of this lane's seed (wave 0)
            for (int g0 = w0; g0 < w1; g0 += G) {
                const int wbase = g0 + wave * W;
                const int nw = max(0, min(W, w1 - wbase));
                double f[W][8];
#pragma unroll
                for (int w = 0; w < W; ++w)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        // wave-uniform: keep the frames in scalar registers
                        const double v = a.frames[8 * (int64_t)(wbase + w) + j];
                        f[w][j] = __hiloint2double(
                            __builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
                    }
                double d2[W];
                Scan::run(sx, sy, sz, 64, P, n_valid, true, f, nw,
                          a.offsets + (nw > 0 ? wbase : 0), a.drift, a.lambda,
                          block_rho + (int64_t)t * rrow, 64, a.evals, lds, d2);
#pragma unroll
                for (int w = 0; w < W; ++w)
                    dd[(wave * W + w) * 64 + lane] = d2[w];
                __syncthreads();
                if (wave == 0) {
                    const int ng = min(G, w1 - g0);
                    for (int j = 0; j < ng; ++j)
                        acc = acc + dd[j * 64 + lane];
                }
                __syncthreads();
            }
            if (wave == 0 && lane < n_valid)
                a.rss[(int64_t)p * a.S + s0 + lane] = acc;
        }

        // Completion counter of partition p; the block that finishes the partition's
        // last tile selects its best seed (Sec. 2.1) while other blocks keep scanning.
        // Wave 0 wrote this item's RSS: its release fence (device scope: the 8 XCDs'
        // L2 caches are not coherent with each other) orders them before its count.
        // The selecting block's acquire fence orders the count before its reads of
        // every tile's RSS. Release fences only write back; the L2 invalidation of
        // an acquire happens once per partition, not once per item.
        if (wave == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const int old = atomicAdd(a.done + p, lane == 0 ? n_sub : 0);
            last_s = n_sub > 0 && __builtin_amdgcn_readfirstlane(old) + n_sub == a.tiles;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(last_s)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int64_t b = block_argmin_n<64 * NWV>(a.rss + (int64_t)p * a.S, a.S);
            if (wave == 0)  // every lane of wave 0 holds the result
                a.best[p] = b;
        }
        __syncthreads();
    }
}

// The wide form, wave-persistent: every wave on its own takes work items (a partition
// and one 64-seed tile) from the work counter, records the tile's tracks into its own
// scratch rows, then scans them against the event's wires W at a time in wire order
// (cdev::TileScanWide; the frames of each group go to the wave's own LDS rows), and
// adds the d^2 of each wire to its lanes' RSS as they come, so the sum runs in wire
// order as in the single-event path. No block barrier: a wave that finishes a
// partition's last tile selects its best seed on its own. WPE: waves per SIMD the
// registers are sized for.
//
// AZ: the wires are taken in azimuth order within the event (the order of the
// single-event wide form: a wave's wires then need nearly the same track chunks), each
// wire's d^2 goes to the wave's own rows and the tile's RSS is summed from them in wire
// order at the end, so that every sum is the same as in wire order. The rows lie in the
// half of the scratch that shapes of at most kMaxBatchNwv / 2 waves leave unused (one
// tile's room per wave: 3 (K + 1) + the radius rows, at least 3 (K + 1) wires); an event
// with more wires takes them in wire order. EXACT: the scan tracks the first index of
// each minimum point by point (no rescan at the end).
template <int W, int NWV, int SUP, int WPE, bool FIELD = false, bool CAP = false,
          bool AZ = false, bool EXACT = false, int HS = 0, bool BLK = false>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(WPE))) void
batch_wide_kernel(BatchArgs a)
{
    static_assert(!AZ || 2 * NWV <= kMaxBatchNwv, "the d^2 rows need the scratch's other half");
    __shared__ __align__(16) double fl_all[NWV * W * 8];
    __shared__ double rmax_all[NWV * W];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *const fl = fl_all + wave * W * 8;
    double *const rmx = rmax_all + wave * W;
    const int P = a.K + 1;
    const int64_t row = (int64_t)P * 64;                 // one coordinate of one tile
    const int64_t rrow = (int64_t)radius_rows(P) * 64;  // chunk radii and longest step of one tile
    double *const sx = a.scratch + ((int64_t)blockIdx.x * NWV + wave) * (3 * row + rrow);
    double *const sy = sx + row, *const sz = sy + row;
    double *const rho = sz + row;
    // BLK: a tile is a 2 x 2 x 4 x 4 block of the grid (the four axes, the last fastest)
    // when the axes allow it, so that its 64 tracks stay closer together than those of
    // 64 consecutive seeds (fewer chunks pass the bound); every tile is then full. Lane
    // l of tile t takes seed seed_at(64 t + l), and its RSS goes to that seed's place.
    const bool blk = BLK && a.n0 % 2 == 0 && a.n1 % 2 == 0 && a.n2 % 4 == 0 && a.n3 % 4 == 0;
    auto seed_at = [&](int64_t c) -> int64_t {
        if (!blk)
            return c;
        int64_t r = c >> 6;
        const int l = (int)(c & 63);
        const int b3 = (int)(r % (a.n3 >> 2));
        r /= a.n3 >> 2;
        const int b2 = (int)(r % (a.n2 >> 2));
        r /= a.n2 >> 2;
        const int b1 = (int)(r % (a.n1 >> 1));
        r /= a.n1 >> 1;
        const int64_t i0 = 2 * r + (l >> 5);
        const int i1 = 2 * b1 + ((l >> 4) & 1), i2 = 4 * b2 + ((l >> 2) & 3), i3 = 4 * b3 + (l & 3);
        return ((i0 * a.n1 + i1) * a.n2 + i2) * a.n3 + i3;
    };

    for (;;) {
        const int64_t item = __builtin_amdgcn_readfirstlane(atomicAdd(a.counter, lane == 0 ? 1 : 0));
        if (item >= a.n_items)
            break;
        const int p = (int)(item / a.tiles);
        const int t = (int)(item - (int64_t)p * a.tiles);
        const int64_t s0 = (int64_t)t * 64;
        const int n_valid = (int)min((int64_t)64, a.S - s0);
        const int e = a.part_event[p];
        if (a.active && a.active[e] == 0)
            continue;  // wave-uniform: the partition keeps best -1
        const int w0 = a.ev_wires[e], w1 = a.ev_wires[e + 1];
        if (lane < n_valid) {
            double st[6];
            seed_from_grid(a.grids + 14 * (int64_t)p, a.n0, a.n1, a.n2, a.n3, seed_at(s0 + lane),
                           st);
            if constexpr (FIELD) {
                record_field_track(a.fm, st, a.charge, a.h, a.K, sx, sy, sz, rho + lane, lane);
            } else {
                ChunkRadius rad;
                double x = st[0], y = st[1], z = st[2], px = st[3], py = st[4];
                const StepConsts kc = step_consts(px, py, st[5], a.bz, a.charge, a.h);
                for (int k = 0; k < a.K; ++k) {
                    sx[(int64_t)k * 64 + lane] = x;
                    sy[(int64_t)k * 64 + lane] = y;
                    sz[(int64_t)k * 64 + lane] = z;
                    rad.add(k, P, x, y, z, rho + lane, 64);
                    rk4_step(kc, x, y, z, px, py);
                }
                sx[(int64_t)a.K * 64 + lane] = x;
                sy[(int64_t)a.K * 64 + lane] = y;
                sz[(int64_t)a.K * 64 + lane] = z;
                rad.add(a.K, P, x, y, z, rho + lane, 64);
            }
        }
        // each lane reads back only its own column; the fence orders its stores before
        // the scan's loads
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        double acc = 0.0;
        const int64_t tile_room = 3 * row + rrow;  // doubles of one tile's scratch
        const bool az = AZ && (int64_t)(w1 - w0) * 64 <= tile_room;  // wave-uniform
        double *const dq =
            AZ ? a.scratch + ((int64_t)kMaxBatchBlocks * NWV + (int64_t)blockIdx.x * NWV + wave) *
                                 tile_room
               : nullptr;
        const double *const frames = az ? a.frames_az : a.frames;
        for (int g0 = w0; g0 < w1; g0 += W) {
            const int nw = min(W, w1 - g0);  // wave-uniform
            // the group's frames into this wave's LDS rows (zero frames past the event)
            for (int i = lane; i < W * 8; i += 64)
                fl[i] = i < nw * 8 ? frames[8 * (int64_t)g0 + i] : 0.0;
            if (CAP && lane < W) {
                // each wire's largest drift distance (-1 without hits), for the cap
                double r = -1.0;
                if (lane < nw) {
                    if (az)
                        r = a.caps_az[g0 + lane];
                    else
                        for (int j = a.offsets[g0 + lane]; j < a.offsets[g0 + lane + 1]; ++j)
                            r = a.drift[j] > r ? a.drift[j] : r;
                }
                rmx[lane] = r;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            int32_t wire_of[W];
#pragma unroll
            for (int w = 0; w < W; ++w)
                wire_of[w] = az && w < nw ? a.wire_of_az[g0 + w] : g0 + w;
            double d2[W];
            TileScanWide<W, SUP, true, CAP, EXACT, HS>::run(sx, sy, sz, 64, P, n_valid, fl, nw,
                                                        wire_of, a.offsets, a.drift, a.lambda,
                                                        rho, 64, a.evals, d2, rmx);
            if (az) {
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (w < nw)
                        dq[(int64_t)(wire_of[w] - w0) * 64 + lane] = d2[w];
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (w < nw)
                        acc = acc + d2[w];
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // frames read before reuse
        }
        if (az)  // each lane reads back its own column, in wire order
            for (int i = 0; i < w1 - w0; ++i)
                acc = acc + dq[(int64_t)i * 64 + lane];
        if (lane < n_valid)
            a.rss[(int64_t)p * a.S + seed_at(s0 + lane)] = acc;
        // completion counter of partition p; the wave that counts its last tile selects
        // the partition's best seed (release before the count, acquire before the reads)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int old = __builtin_amdgcn_readfirstlane(atomicAdd(a.done + p, lane == 0 ? 1 : 0));
        if (old + 1 == a.tiles) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int64_t b = wave_argmin(a.rss + (int64_t)p * a.S, a.S);
            if (lane == 0)
                a.best[p] = b;
        }
    }
}

__global__ void batch_refine_kernel(int n_part, double *__restrict__ grids, int n0, int n1, int n2,
                                    int n3, const int64_t *__restrict__ best)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_part)
        refine_grid_desc(grids + 14 * (int64_t)p, n0, n1, n2, n3, best[p]);
}

// One block per partition: the chosen seed (its descriptor and index), its RSS, and the
// classification of its event's hits (Sec. 2.1): per wire the hit with the smallest
// |D - r_j| (first on ties) gets bit 0 when below lambda and bit 1 within 1e-9 mm of
// lambda. The seed's track is recomputed into LDS (thread 0).
constexpr int kBatchClassifyThreads = 256;

__global__ __launch_bounds__(kBatchClassifyThreads) void batch_classify_kernel(
    const double *__restrict__ grids, int n0, int n1, int n2, int n3, int64_t S,
    const int64_t *__restrict__ best, const double *__restrict__ rss,
    const double *__restrict__ ends, const int32_t *__restrict__ offsets,
    const double *__restrict__ drift, const int32_t *__restrict__ ev_wires,
    const int32_t *__restrict__ part_event, double bz, double charge, double h, int K,
    double lambda, double *__restrict__ best_seed, double *__restrict__ best_rss,
    uint8_t *__restrict__ mask, int64_t mask_stride, int32_t *__restrict__ n_border,
    FieldMap fm, int use_field)
{
    extern __shared__ double pts[];  // [3][K + 1]
    __shared__ int32_t border;
    const int p = blockIdx.x;
    const int P = K + 1;
    const int64_t b = best[p];
    const int e = part_event[p];
    const int w0 = ev_wires[e], w1 = ev_wires[e + 1];
    const int h0 = offsets[w0];
    if (threadIdx.x == 0) {
        border = 0;
        double st[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
        if (b >= 0 && use_field) {
            seed_from_grid(grids + 14 * (int64_t)p, n0, n1, n2, n3, b, st);
            // the steps of rk4_field_record_kernel (RK4, or RKN for fm.stepper 1)
            double x[3] = {st[0], st[1], st[2]}, q[3] = {st[3], st[4], st[5]};
            const double p0 = sqrt((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
            const double inv = 1.0 / p0;
            const double g = (kKappa * charge) * inv;
            const bool rkn = fm.stepper == 1;
            const RknConsts kn = rkn_consts(h);
            if (rkn)
                for (int c = 0; c < 3; ++c)
                    q[c] = q[c] * inv;
            for (int k = 0; k < K; ++k) {
                pts[k] = x[0];
                pts[P + k] = x[1];
                pts[2 * P + k] = x[2];
                if (rkn)
                    rkn_field_step(fm, kn, g, x, q);
                else
                    rk4_field_step(fm, inv, g, h, x, q);
            }
            pts[K] = x[0];
            pts[P + K] = x[1];
            pts[2 * P + K] = x[2];
        } else if (b >= 0) {
            seed_from_grid(grids + 14 * (int64_t)p, n0, n1, n2, n3, b, st);
            double x = st[0], y = st[1], z = st[2], px = st[3], py = st[4];
            const StepConsts kc = step_consts(px, py, st[5], bz, charge, h);
            for (int k = 0; k < K; ++k) {
                pts[k] = x;
                pts[P + k] = y;
                pts[2 * P + k] = z;
                rk4_step(kc, x, y, z, px, py);
            }
            pts[K] = x;
            pts[P + K] = y;
            pts[2 * P + K] = z;
        }
        if (best_seed)
            for (int c = 0; c < 6; ++c)
                best_seed[6 * (int64_t)p + c] = st[c];
        if (best_rss)
            best_rss[p] = b >= 0 ? rss[(int64_t)p * S + b] : NAN;
    }
    __syncthreads();
    for (int wi = w0 + threadIdx.x; wi < w1; wi += kBatchClassifyThreads) {
        const int j0 = offsets[wi], j1 = offsets[wi + 1];
        uint8_t *m = mask ? mask + (int64_t)p * mask_stride - h0 : nullptr;
        if (m)
            for (int j = j0; j < j1; ++j)
                m[j] = 0;
        if (b < 0)
            continue;
        double f[8];
        wire_frame(ends + 6 * (int64_t)wi, f);
        double qb = INFINITY;
        int kb = 0;
        for (int k = 0; k < P; ++k) {
            double xi, eta;
            project(f, pts[k], pts[P + k], pts[2 * P + k], xi, eta);
            const double q = fma(xi, xi, eta * eta);
            if (q < qb) {
                qb = q;
                kb = k;
            }
        }
        const double D = sqrt(refine_dca2(pts, pts + P, pts + 2 * P, 1, P, f, kb, qb));
        int jb = -1;
        double eb = INFINITY;
        for (int j = j0; j < j1; ++j) {
            const double r = fabs(D - drift[j]);
            if (r < eb) {
                eb = r;
                jb = j;
            }
        }
        if (jb >= 0) {
            uint8_t bits = 0;
            if (eb < lambda)
                bits |= 1;
            if (fabs(eb - lambda) < 1e-9) {
                bits |= 2;
                atomicAdd(&border, 1);  // LDS counter: integer, order-independent
            }
            if (m)
                m[jb] = bits;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && n_border)
        n_border[p] = border;
}

// k smallest (value, index) pairs of each segment in increasing order (ties: lower
// index; NaN never chosen; -1 when fewer than k values are not NaN). Round r takes the
// smallest pair strictly above round r-1's, so no membership test is needed.
__global__ __launch_bounds__(kSelectThreads) void topk_kernel(const double *__restrict__ v,
                                                              int64_t n, int k,
                                                              int64_t *__restrict__ out)
{
    __shared__ double sv[kSelectThreads / 64];
    __shared__ int64_t si[kSelectThreads / 64];
    __shared__ double prev_v;
    __shared__ int64_t prev_i;
    const double *seg = v + (int64_t)blockIdx.x * n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        prev_v = -INFINITY;
        prev_i = -1;
    }
    __syncthreads();
    for (int r = 0; r < k; ++r) {
        const double pv = prev_v;
        const int64_t pi = prev_i;
        MinLoc m{INFINITY, -1};
        for (int64_t s = threadIdx.x; s < n; s += kSelectThreads) {
            const double x = seg[s];
            const bool above = x > pv || (x == pv && s > pi);  // NaN is never above
            if (above && (x < m.v || (m.i < 0 && x == m.v))) {
                m.v = x;
                m.i = s;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            MinLoc o{__shfl_xor(m.v, off), __shfl_xor(m.i, off)};
            if (beats(o, m))
                m = o;
        }
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
            if (lane == 0) {
                out[(int64_t)blockIdx.x * k + r] = a.i;
                if (a.i >= 0) {
                    prev_v = a.v;
                    prev_i = a.i;
                } else {
                    prev_v = NAN;  // nothing is above NaN: later rounds give -1
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ several references
// Sec. 2.1: several low-RSS seeds become reference points of the next, finer scan,
// sparse enough that the new seed sets around them do not overlap. A candidate is a
// seed (u, i) of one of a group's n_sub grids; its new seed set is the box centred on
// its axis values with the refined half-spans 2 half / (n - 1) (the grid's own centre
// and half-span on an axis with n = 1). Boxes overlap when on every axis the centres
// are equal or fabs(c1 - c2) < 0.999999999 * (h1 + h2) (the factor keeps boxes that
// only touch apart whatever the rounding). Greedy in increasing (rss, candidate
// index): a candidate is taken when its box overlaps none taken before.
constexpr int kMaxRefs = 64;

__device__ __forceinline__ void candidate_box(const double *__restrict__ g, const int (&n)[4],
                                              int64_t i, double (&c)[4], double (&h)[4])
{
    int idx[4];
    int64_t rest = i;
    for (int a = 3; a >= 0; --a) {
        idx[a] = (int)(rest % n[a]);
        rest /= n[a];
    }
    for (int a = 0; a < 4; ++a) {
        if (n[a] > 1) {
            c[a] = axis_value(g[6 + a], g[10 + a], n[a], idx[a]);
            h[a] = (2.0 * g[10 + a]) / (double)(n[a] - 1);
        } else {
            c[a] = g[6 + a];
            h[a] = g[10 + a];
        }
    }
}

__device__ __forceinline__ bool boxes_overlap(const double (&c1)[4], const double (&h1)[4],
                                              const double *c2, const double *h2)
{
    for (int a = 0; a < 4; ++a)
        if (!(c1[a] == c2[a] || fabs(c1[a] - c2[a]) < 0.999999999 * (h1[a] + h2[a])))
            return false;
    return true;
}

// One block per group. Each round, every thread finds its lowest (rss, index)
// candidate whose box is free, the block reduces to the winner and wave 0 records it.
// Control flow around the barriers is block-uniform (the winner comes from LDS).
__global__ __launch_bounds__(kSelectThreads) void sparse_select_kernel(
    const double *__restrict__ grids, const double *__restrict__ rss, int n_sub, int n0, int n1,
    int n2, int n3, int64_t S, int n_ref, int64_t *__restrict__ ref_idx,
    double *__restrict__ ref_rss, double *__restrict__ new_grids, double *__restrict__ ref_grids,
    int64_t *__restrict__ ref_local)
{
    __shared__ double tc[kMaxRefs][4], th[kMaxRefs][4];
    __shared__ double wv[kSelectThreads / 64];
    __shared__ int64_t wi[kSelectThreads / 64];
    __shared__ double win_v;
    __shared__ int64_t win_i;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n[4] = {n0, n1, n2, n3};
    const int64_t grp = blockIdx.x;
    const double *gg = grids + 14 * grp * n_sub;
    const double *rr = rss + grp * n_sub * S;
    const int64_t total = S * n_sub;
    const int64_t out0 = grp * n_ref;
    int taken = 0;
    for (int r = 0; r < n_ref; ++r) {
        MinLoc m{INFINITY, -1};
        for (int64_t j = threadIdx.x; j < total; j += kSelectThreads) {
            const double v = rr[j];
            if (!(v < m.v || (m.i < 0 && v == m.v)))
                continue;  // not better than this thread's best so far (NaN never is)
            double c[4], h[4];
            candidate_box(gg + 14 * (j / S), n, j % S, c, h);
            bool free_box = true;
            for (int t = 0; t < taken && free_box; ++t)
                if (boxes_overlap(c, h, tc[t], th[t]))
                    free_box = false;
            if (free_box) {
                m.v = v;
                m.i = j;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            MinLoc o{__shfl_xor(m.v, off), __shfl_xor(m.i, off)};
            if (beats(o, m))
                m = o;
        }
        if (lane == 0) {
            wv[wave] = m.v;
            wi[wave] = m.i;
        }
        __syncthreads();
        if (wave == 0) {
            MinLoc a{INFINITY, -1};
            if (lane < kSelectThreads / 64) {
                a.v = wv[lane];
                a.i = wi[lane];
            }
            for (int off = 32; off > 0; off >>= 1) {
                MinLoc o{__shfl_xor(a.v, off), __shfl_xor(a.i, off)};
                if (beats(o, a))
                    a = o;
            }
            if (lane == 0) {
                win_v = a.v;
                win_i = a.i;
            }
        }
        __syncthreads();
        const int64_t j = __builtin_amdgcn_readfirstlane((int)win_i);  // < 2^31 (host check)
        if (j < 0)
            break;
        if (wave == 0 && lane == 0) {
            const double *g = gg + 14 * (j / S);
            double c[4], h[4];
            candidate_box(g, n, j % S, c, h);
            for (int a = 0; a < 4; ++a) {
                tc[taken][a] = c[a];
                th[taken][a] = h[a];
            }
            ref_idx[out0 + r] = j;
            if (ref_rss)
                ref_rss[out0 + r] = win_v;
            if (ref_local)
                ref_local[out0 + r] = j % S;
            double d[14];
            for (int q = 0; q < 14; ++q)
                d[q] = g[q];
            if (ref_grids)
                for (int q = 0; q < 14; ++q)
                    ref_grids[14 * (out0 + r) + q] = d[q];
            refine_grid_desc(d, n0, n1, n2, n3, j % S);
            for (int q = 0; q < 14; ++q)
                new_grids[14 * (out0 + r) + q] = d[q];
        }
        __syncthreads();
        ++taken;
    }
    // past the last reference: -1, NaN and copies of reference 0 (of grid 0 if none)
    for (int r = taken; r < n_ref; ++r) {
        if (threadIdx.x == 0) {
            ref_idx[out0 + r] = -1;
            if (ref_rss)
                ref_rss[out0 + r] = NAN;
            if (ref_local)
                ref_local[out0 + r] = -1;
        }
        if (threadIdx.x < 14) {
            const int q = threadIdx.x;
            new_grids[14 * (out0 + r) + q] = taken > 0 ? new_grids[14 * out0 + q] : gg[q];
            if (ref_grids)
                ref_grids[14 * (out0 + r) + q] = taken > 0 ? ref_grids[14 * out0 + q] : gg[q];
        }
    }
}

// Seeds at chosen grid indices: out[:, p k + r] = seed idx[p k + r] of grids[p]
// (NaN for idx < 0). One thread per (partition, rank).
__global__ void grid_seeds_kernel(const double *__restrict__ grids, int n0, int n1, int n2, int n3,
                                  const int64_t *__restrict__ idx, int n_part, int k,
                                  double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_part * k;
    if (t >= total)
        return;
    const int p = (int)(t / k);
    double st[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
    if (idx[t] >= 0)
        seed_from_grid(grids + 14 * (int64_t)p, n0, n1, n2, n3, idx[t], st);
    for (int c = 0; c < 6; ++c)
        out[c * total + t] = st[c];
}

__global__ void batch_frames_kernel(const double *__restrict__ ends, int n_w, int n_pad,
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
        // the azimuth of the wire's midpoint; a NaN endpoint sorts after every azimuth
        k = atan2f((float)(e[1] + e[4]), (float)(e[0] + e[3]));
        if (k != k)
            k = 4.0f;
    }
    for (int j = 0; j < 8; ++j)
        frames[8 * (int64_t)w + j] = f[j];
    key[w] = k;
}

// The wires of each event in azimuth order: wire i of event e goes to slot w0 + its rank
// among the event's wires in (key, index) order, with its frame and its largest drift
// distance (-1 without hits). Only the wires of the events are touched.
__global__ void batch_wire_order_kernel(const double *__restrict__ frames,
                                        const float *__restrict__ key,
                                        const int32_t *__restrict__ ev_wires, int n_events,
                                        const int32_t *__restrict__ offsets,
                                        const double *__restrict__ drift,
                                        double *__restrict__ frames_az,
                                        int32_t *__restrict__ wire_of_az,
                                        double *__restrict__ caps_az)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ev_wires[n_events] || i < ev_wires[0])
        return;
    int lo = 0, hi = n_events;  // the event e with ev_wires[e] <= i < ev_wires[e + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (ev_wires[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    const int w0 = ev_wires[lo], w1 = ev_wires[lo + 1];
    const float ki = key[i];
    int rank = 0;
    for (int j = w0; j < w1; ++j) {
        const float kj = key[j];
        rank += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
    }
    const int r = w0 + rank;
    for (int j = 0; j < 8; ++j)
        frames_az[8 * (int64_t)r + j] = frames[8 * (int64_t)i + j];
    wire_of_az[r] = i;
    double rmax = -1.0;
    for (int j = offsets[i]; j < offsets[i + 1]; ++j)
        rmax = drift[j] > rmax ? drift[j] : rmax;
    caps_az[r] = rmax;
}

// Start of a scan: empty work queue, no tile finished, no partition selected yet.
__global__ void reset_scan_kernel(int *counter, int *done, int64_t *best, int n_part)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0)
        *counter = 0;
    if (p < n_part) {
        done[p] = 0;
        best[p] = -1;
    }
}

__global__ void copy_kernel(const double *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ shapes
struct BatchVariant {
    int w, nwv, c, direct;  // direct: 0 LDS-staged, 1 every wave on its own, 2 wide
    void (*kernel)(BatchArgs);
    int runs;  // direct and wide shapes: chunks tested in runs of this many first (1: no runs)
};

const BatchVariant kBatchVariants[] = {
    {4, 8, 16, 0, batch_scan_kernel<4, 8, 16, 4, false>},
    {3, 8, 16, 0, batch_scan_kernel<3, 8, 16, 4, false>},
    {2, 8, 16, 0, batch_scan_kernel<2, 8, 16, 4, false>},
    {4, 8, 16, 0, batch_scan_kernel<4, 8, 16, 1, false>},
    {5, 8, 16, 0, batch_scan_kernel<5, 8, 16, 1, false>},
    {6, 8, 16, 0, batch_scan_kernel<6, 8, 16, 1, false>},
    // every wave on its own (no LDS staging)
    {4, 8, 16, 1, batch_scan_kernel<4, 8, 16, 4, true>},
    {3, 8, 16, 1, batch_scan_kernel<3, 8, 16, 4, true>},
    {2, 8, 16, 1, batch_scan_kernel<2, 8, 16, 4, true>},
    // runs of 4 chunks tested first (two-level distance bound)
    {4, 8, 16, 1, batch_scan_kernel<4, 8, 16, 4, true, false, 4>, 4},
    {3, 8, 16, 1, batch_scan_kernel<3, 8, 16, 4, true, false, 4>, 4},
    // wide, wave-persistent: one tile per wave item, W wires per pass in wire order
    {16, 4, 16, 2, batch_wide_kernel<16, 4, 4, 2>, 4},
    {16, 4, 16, 2, batch_wide_kernel<16, 4, 1, 2>, 1},
    {12, 4, 16, 2, batch_wide_kernel<12, 4, 4, 2>, 4},
    // wide with the residual cap in the bound (direct == 3)
    {16, 4, 16, 3, batch_wide_kernel<16, 4, 4, 2, false, true>, 4},
    {12, 4, 16, 3, batch_wide_kernel<12, 4, 4, 2, false, true>, 4},
    {8, 4, 16, 3, batch_wide_kernel<8, 4, 4, 2, false, true>, 4},
    // wide with the cap, wires in azimuth order within each event (direct == 4)
    {16, 4, 16, 4, batch_wide_kernel<16, 4, 4, 2, false, true, true>, 4},
    {12, 4, 16, 4, batch_wide_kernel<12, 4, 4, 2, false, true, true>, 4},
    {8, 4, 16, 4, batch_wide_kernel<8, 4, 4, 2, false, true, true>, 4},
    // the same with the first index of the minimum tracked point by point (direct == 5)
    {16, 4, 16, 5, batch_wide_kernel<16, 4, 4, 2, false, true, true, true>, 4},
    {12, 4, 16, 5, batch_wide_kernel<12, 4, 4, 2, false, true, true, true>, 4},
    // ... with each half (or quarter) of a needed chunk tested per wire, every test from
    // the middle of its stretch (on the full 1024-event mix: 196 events/s for 12 wires
    // in halves, 183 for 16; 16 wires in quarters 183, 8 wires in halves 175)
    {16, 4, 16, 5, batch_wide_kernel<16, 4, 4, 2, false, true, true, true, 2>, 4},
    {12, 4, 16, 5, batch_wide_kernel<12, 4, 4, 2, false, true, true, true, 2>, 4},
    {12, 4, 16, 5, batch_wide_kernel<12, 4, 4, 2, false, true, true, true, 4>, 4},
    // ... with each tile a 2 x 2 x 4 x 4 block of the grid
    {12, 4, 16, 5, batch_wide_kernel<12, 4, 4, 2, false, true, true, true, 2, true>, 4},
    {16, 4, 16, 5, batch_wide_kernel<16, 4, 4, 2, false, true, true, true, 2, true>, 4},
};
constexpr int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);
// Tracks in a field map: one shape (the wave-independent 4 x 8 x 16), so the uniform
// kernels above keep their registers.
const BatchVariant kBatchFieldVariant = {4, 8, 16, 1, batch_scan_kernel<4, 8, 16, 4, true, true>};


std::mutex g_batch_mu;
int g_batch_variant = 0;
// persistent grid per (variant, device); the last row is the field-map kernel's
int g_batch_blocks[kNumBatchVariants + 1][64];

const BatchVariant &batch_variant(int id)
{
    return id < kNumBatchVariants ? kBatchVariants[id] : kBatchFieldVariant;
}

// Persistent blocks for a shape: every block that can be resident at once.
int batch_blocks(int id)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    std::lock_guard<std::mutex> lock(g_batch_mu);
    int &nb = g_batch_blocks[id][dev];
    if (nb == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        const BatchVariant &v = batch_variant(id);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)v.kernel,
                                                         64 * v.nwv, 0) != hipSuccess)
            return 0;
        nb = min(kMaxBatchBlocks, max(1, cus * max(1, per_cu)));
    }
    return nb;
}

// Scratch of one persistent block: the tracks and chunk radii of kMaxBatchNwv tiles of
// 64 seeds.
size_t batch_scratch_bytes(int K)
{
    return sizeof(double) * (3 * (size_t)(K + 1) + (size_t)radius_rows(K + 1)) * 64 *
           kMaxBatchNwv;
}

int frames_pad(int n_w) { return ((n_w + 63) / 64) * 64 + kBatchWirePad; }

struct BatchLayout {
    double *frames;
    int *counter;
    int *done;
    double *scratch;
    float *key;
    double *frames_az;
    int32_t *wire_of_az;
    double *caps_az;
};

BatchLayout batch_layout(void *ws, int n_wires, int n_partitions, int K)
{
    char *p = (char *)ws;
    const size_t pad = (size_t)frames_pad(n_wires);
    BatchLayout l;
    l.frames = (double *)p;
    p += align256(sizeof(double) * 8 * pad);
    l.counter = (int *)p;
    p += 256;
    l.done = (int *)p;
    p += align256(sizeof(int) * (size_t)n_partitions);
    l.scratch = (double *)p;
    p += (size_t)kMaxBatchBlocks * batch_scratch_bytes(K);
    l.key = (float *)p;
    p += align256(sizeof(float) * pad);
    l.frames_az = (double *)p;
    p += align256(sizeof(double) * 8 * pad);
    l.wire_of_az = (int32_t *)p;
    p += align256(sizeof(int32_t) * pad);
    l.caps_az = (double *)p;
    return l;
}

// The device view of a caller's field map (an empty map, unused, when there is none).
FieldMap field_map(const comet_field *f)
{
    if (!f)
        return FieldMap{nullptr, 0, 0, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 0};
    return FieldMap{f->b, f->nx, f->ny, f->nz, f->x0, f->y0, f->z0, f->dx, f->dy, f->dz,
                    f->stepper};
}

int launch_batch_classify(const double *grids, int n_partitions, const int32_t n[4], int64_t S,
                          const int64_t *best, const double *rss, const double *wire_ends,
                          const int32_t *wire_offsets, const double *drift,
                          const int32_t *event_wires, const int32_t *part_event,
                          const comet_config *cfg, double *best_seed, double *best_rss,
                          uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                          const comet_field *field, hipStream_t hs)
{
    const size_t lds = sizeof(double) * 3 * (size_t)(cfg->n_steps + 1);
    hipLaunchKernelGGL(batch_classify_kernel, dim3(n_partitions), dim3(kBatchClassifyThreads), lds,
                       hs, grids, n[0], n[1], n[2], n[3], S, best, rss, wire_ends, wire_offsets,
                       drift, event_wires, part_event, cfg->bz_tesla, cfg->charge_e,
                       cfg->step_mm, cfg->n_steps, cfg->lambda_mm, best_seed, best_rss, hit_mask,
                       mask_stride, n_borderline, field_map(field), field ? 1 : 0);
    return launched("batch_classify_kernel");
}

}  // namespace

extern "C" {

size_t comet_batch_workspace_bytes(int32_t n_wires, int32_t n_steps, int32_t n_partitions)
{
    if (n_wires < 0 || n_steps < 1 || n_partitions < 0)
        return 0;
    const size_t pad = (size_t)frames_pad(n_wires);
    return align256(sizeof(double) * 8 * pad) + 256 +
           align256(sizeof(int) * (size_t)n_partitions) +
           (size_t)kMaxBatchBlocks * batch_scratch_bytes(n_steps) + align256(sizeof(float) * pad) +
           align256(sizeof(double) * 8 * pad) + align256(sizeof(int32_t) * pad) +
           align256(sizeof(double) * pad);
}

}  // extern "C"

namespace {

int batch_scan_impl(const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                    const double *drift, int32_t n_hits, const int32_t *event_wires,
                    int32_t n_events, const int32_t *part_event, int32_t n_partitions,
                    const double *grids_init, double *grids, const int32_t n[4],
                    const comet_config *cfg, const comet_field *field, int32_t n_refine,
                    double *rss, int64_t *best, double *best_seed, double *best_rss,
                    uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                    int64_t max_items, void *workspace, size_t workspace_bytes, void *stream,
                    const int32_t *event_active = nullptr)
{
    if (!wire_ends || !wire_offsets || !event_wires || !part_event || !grids || !n || !rss ||
        !best)
        return fail(COMET_EINVAL, "comet_batch_scan: NULL pointer");
    if (n_wires < 1 || n_hits < 0 || (n_hits > 0 && !drift) || n_events < 1 || n_partitions < 1)
        return fail(COMET_EINVAL, "comet_batch_scan: bad sizes");
    if (n_refine < 0 || n_refine > 100)
        return fail(COMET_EINVAL, "comet_batch_scan: n_refine must be in [0, 100]");
    int64_t S = 1;
    for (int a = 0; a < 4; ++a) {
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_batch_scan: n[%d] < 1", a);
        S *= n[a];
    }
    if (S > ((int64_t)1 << 31) ||
        (int64_t)n_partitions * ((S + 63) / 64) + kMaxBatchBlocks > ((int64_t)1 << 31) - 1 ||
        (int64_t)n_partitions * ((S + 63) / 64) > ((int64_t)1 << 31) - 1)
        return fail(COMET_EINVAL, "comet_batch_scan: too many work items for one launch");
    int st = check_config(cfg);
    if (st)
        return st;
    if (cfg->n_steps > 2400)
        return fail(COMET_EUNSUPPORTED, "comet_batch_scan: n_steps %d > 2400", cfg->n_steps);
    if (hit_mask && mask_stride < 1)
        return fail(COMET_EINVAL, "comet_batch_scan: mask_stride must be >= 1");
    const size_t need = comet_batch_workspace_bytes(n_wires, cfg->n_steps, n_partitions);
    if (!workspace || workspace_bytes < need)
        return fail(COMET_EWORKSPACE, "comet_batch_scan: workspace %zu < %zu bytes",
                    workspace_bytes, need);
    if (((uintptr_t)workspace & 255) != 0)
        return fail(COMET_EINVAL, "comet_batch_scan: workspace not 256-byte aligned");
    st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    const BatchLayout l = batch_layout(workspace, n_wires, n_partitions, cfg->n_steps);
    if (grids_init) {
        const int64_t nd = 14 * (int64_t)n_partitions;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, hs,
                           grids_init, grids, nd);
        st = launched("copy_kernel");
        if (st)
            return st;
    }
    const int pad = frames_pad(n_wires);
    hipLaunchKernelGGL(batch_frames_kernel, dim3((pad + 63) / 64), dim3(64), 0, hs, wire_ends,
                       n_wires, pad, l.frames, l.key);
    st = launched("batch_frames_kernel");
    if (st)
        return st;
    int id;
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        id = g_batch_variant;
    }
    if (field)
        id = kNumBatchVariants;  // the field-map kernel
    const BatchVariant &v = batch_variant(id);
    if (v.direct >= 4) {
        hipLaunchKernelGGL(batch_wire_order_kernel, dim3((n_wires + 255) / 256), dim3(256), 0, hs,
                           (const double *)l.frames, (const float *)l.key, event_wires, n_events,
                           wire_offsets, drift, l.frames_az, l.wire_of_az, l.caps_az);
        st = launched("batch_wire_order_kernel");
        if (st)
            return st;
    }
    const int blocks = batch_blocks(id);
    if (blocks < 1)
        return fail(COMET_EHIP, "comet_batch_scan: occupancy query failed");
    const int tiles = (int)((S + 63) / 64);
    const int per_item = v.direct >= 2 ? 1 : v.nwv;  // tiles per work item (wide: one)
    const int supers = (tiles + per_item - 1) / per_item;
    int64_t max_tiles = (int64_t)n_partitions * tiles;
    if (max_items > 0 && max_items < max_tiles)
        max_tiles = max_items;
    // work items: the super-tiles that hold at least one of the first max_tiles tiles
    const int64_t full = max_tiles / tiles, rest = max_tiles - full * tiles;
    const int64_t items = full * supers + (rest + per_item - 1) / per_item;
    BatchArgs args{l.frames, wire_offsets, drift, event_wires, part_event, grids, n[0], n[1],
                   n[2], n[3], S, tiles, supers, items, max_tiles, cfg->bz_tesla,
                   cfg->charge_e, cfg->step_mm, cfg->lambda_mm, cfg->n_steps, l.scratch,
                   l.counter, l.done, rss, best, scan_counter(), field_map(field), event_active,
                   l.frames_az, l.wire_of_az, l.caps_az};
    for (int it = 0; it <= n_refine && st == COMET_OK; ++it) {
        if (it) {
            hipLaunchKernelGGL(batch_refine_kernel, dim3((n_partitions + 255) / 256), dim3(256), 0,
                               hs, n_partitions, grids, n[0], n[1], n[2], n[3],
                               (const int64_t *)best);
            st = launched("batch_refine_kernel");
            if (st)
                break;
        }
        hipLaunchKernelGGL(reset_scan_kernel, dim3((n_partitions + 255) / 256), dim3(256), 0, hs,
                           l.counter, l.done, best, n_partitions);
        st = launched("reset_scan_kernel");
        if (st)
            break;
        ProfScope prof(kProfDca, hs);
        hipLaunchKernelGGL(v.kernel, dim3(blocks), dim3(64 * v.nwv), 0, hs, args);
        st = launched("batch_scan_kernel");
    }
    if (st)
        return st;
    if (!best_seed && !best_rss && !hit_mask && !n_borderline)
        return COMET_OK;  // no classification output asked for
    return launch_batch_classify(grids, n_partitions, n, S, best, rss, wire_ends, wire_offsets,
                                 drift, event_wires, part_event, cfg, best_seed, best_rss,
                                 hit_mask, mask_stride, n_borderline, field, hs);
}

int batch_classify_impl(const double *grids, int32_t n_partitions, const int32_t n[4],
                        const int64_t *best, const double *rss, const double *wire_ends,
                        int32_t n_wires, const int32_t *wire_offsets, const double *drift,
                        int32_t n_hits, const int32_t *event_wires, int32_t n_events,
                        const int32_t *part_event, const comet_config *cfg,
                        const comet_field *field, double *best_seed, double *best_rss,
                        uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                        void *stream)
{
    if (!grids || !n || !best || !wire_ends || !wire_offsets || !event_wires || !part_event)
        return fail(COMET_EINVAL, "comet_batch_classify: NULL pointer");
    if (n_partitions < 1 || n_wires < 1 || n_hits < 0 || (n_hits > 0 && !drift) || n_events < 1)
        return fail(COMET_EINVAL, "comet_batch_classify: bad sizes");
    if (best_rss && !rss)
        return fail(COMET_EINVAL, "comet_batch_classify: best_rss needs rss");
    if (hit_mask && mask_stride < 1)
        return fail(COMET_EINVAL, "comet_batch_classify: mask_stride must be >= 1");
    int64_t S = 1;
    for (int a = 0; a < 4; ++a) {
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_batch_classify: n[%d] < 1", a);
        S *= n[a];
    }
    int st = check_config(cfg);
    if (st)
        return st;
    if (cfg->n_steps > 2400)
        return fail(COMET_EUNSUPPORTED, "comet_batch_classify: n_steps %d > 2400", cfg->n_steps);
    st = check_device();
    if (st)
        return st;
    return launch_batch_classify(grids, n_partitions, n, S, best, rss, wire_ends, wire_offsets,
                                 drift, event_wires, part_event, cfg, best_seed, best_rss,
                                 hit_mask, mask_stride, n_borderline, field, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int comet_batch_scan(const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                     const double *drift, int32_t n_hits, const int32_t *event_wires,
                     int32_t n_events, const int32_t *part_event, int32_t n_partitions,
                     const double *grids_init, double *grids, const int32_t n[4],
                     const comet_config *cfg, int32_t n_refine, double *rss, int64_t *best,
                     double *best_seed, double *best_rss, uint8_t *hit_mask,
                     int64_t mask_stride, int32_t *n_borderline, int64_t max_items,
                     void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    return batch_scan_impl(wire_ends, n_wires, wire_offsets, drift, n_hits, event_wires,
                           n_events, part_event, n_partitions, grids_init, grids, n, cfg,
                           nullptr, n_refine, rss, best, best_seed, best_rss, hit_mask,
                           mask_stride, n_borderline, max_items, workspace, workspace_bytes,
                           stream);
}

int comet_batch_scan_active(const double *wire_ends, int32_t n_wires,
                            const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                            const int32_t *event_wires, int32_t n_events,
                            const int32_t *part_event, int32_t n_partitions,
                            const double *grids_init, double *grids, const int32_t n[4],
                            const comet_config *cfg, int32_t n_refine, double *rss,
                            int64_t *best, double *best_seed, double *best_rss,
                            uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                            const int32_t *event_active, void *workspace,
                            size_t workspace_bytes, void *stream)
{
    clear_error();
    if (!event_active)
        return fail(COMET_EINVAL, "comet_batch_scan_active: NULL event_active");
    return batch_scan_impl(wire_ends, n_wires, wire_offsets, drift, n_hits, event_wires,
                           n_events, part_event, n_partitions, grids_init, grids, n, cfg,
                           nullptr, n_refine, rss, best, best_seed, best_rss, hit_mask,
                           mask_stride, n_borderline, 0, workspace, workspace_bytes, stream,
                           event_active);
}

int comet_batch_scan_field(const double *wire_ends, int32_t n_wires,
                           const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                           const int32_t *event_wires, int32_t n_events,
                           const int32_t *part_event, int32_t n_partitions,
                           const double *grids_init, double *grids, const int32_t n[4],
                           const comet_config *cfg, const comet_field *field, int32_t n_refine,
                           double *rss, int64_t *best, double *best_seed, double *best_rss,
                           uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                           int64_t max_items, void *workspace, size_t workspace_bytes,
                           void *stream)
{
    clear_error();
    const int st = check_field("comet_batch_scan_field", field);
    if (st)
        return st;
    return batch_scan_impl(wire_ends, n_wires, wire_offsets, drift, n_hits, event_wires,
                           n_events, part_event, n_partitions, grids_init, grids, n, cfg, field,
                           n_refine, rss, best, best_seed, best_rss, hit_mask, mask_stride,
                           n_borderline, max_items, workspace, workspace_bytes, stream);
}

int comet_batch_classify(const double *grids, int32_t n_partitions, const int32_t n[4],
                         const int64_t *best, const double *rss, const double *wire_ends,
                         int32_t n_wires, const int32_t *wire_offsets, const double *drift,
                         int32_t n_hits, const int32_t *event_wires, int32_t n_events,
                         const int32_t *part_event, const comet_config *cfg, double *best_seed,
                         double *best_rss, uint8_t *hit_mask, int64_t mask_stride,
                         int32_t *n_borderline, void *stream)
{
    clear_error();
    return batch_classify_impl(grids, n_partitions, n, best, rss, wire_ends, n_wires,
                               wire_offsets, drift, n_hits, event_wires, n_events, part_event,
                               cfg, nullptr, best_seed, best_rss, hit_mask, mask_stride,
                               n_borderline, stream);
}

int comet_batch_classify_field(const double *grids, int32_t n_partitions, const int32_t n[4],
                               const int64_t *best, const double *rss, const double *wire_ends,
                               int32_t n_wires, const int32_t *wire_offsets,
                               const double *drift, int32_t n_hits, const int32_t *event_wires,
                               int32_t n_events, const int32_t *part_event,
                               const comet_config *cfg, const comet_field *field,
                               double *best_seed, double *best_rss, uint8_t *hit_mask,
                               int64_t mask_stride, int32_t *n_borderline, void *stream)
{
    clear_error();
    const int st = check_field("comet_batch_classify_field", field);
    if (st)
        return st;
    return batch_classify_impl(grids, n_partitions, n, best, rss, wire_ends, n_wires,
                               wire_offsets, drift, n_hits, event_wires, n_events, part_event,
                               cfg, field, best_seed, best_rss, hit_mask, mask_stride,
                               n_borderline, stream);
}

int comet_sparse_select(const double *grids, const double *rss, int32_t n_groups, int32_t n_sub,
                        const int32_t n[4], int32_t n_ref, int64_t *ref_idx, double *ref_rss,
                        double *new_grids, double *ref_grids, int64_t *ref_local, void *stream)
{
    clear_error();
    if (!grids || !rss || !n || !ref_idx || !new_grids)
        return fail(COMET_EINVAL, "comet_sparse_select: NULL pointer");
    if (n_groups < 1 || n_sub < 1 || n_ref < 1 || n_ref > kMaxRefs)
        return fail(COMET_EINVAL, "comet_sparse_select: need n_groups, n_sub >= 1 and "
                                  "1 <= n_ref <= %d", kMaxRefs);
    int64_t S = 1;
    for (int a = 0; a < 4; ++a) {
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_sparse_select: n[%d] < 1", a);
        S *= n[a];
    }
    if (S * n_sub > ((int64_t)1 << 31) - 1)
        return fail(COMET_EINVAL, "comet_sparse_select: more than 2^31 - 1 candidates a group");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(sparse_select_kernel, dim3(n_groups), dim3(kSelectThreads), 0,
                       (hipStream_t)stream, grids, rss, n_sub, n[0], n[1], n[2], n[3], S, n_ref,
                       ref_idx, ref_rss, new_grids, ref_grids, ref_local);
    return launched("sparse_select_kernel");
}

int comet_topk(const double *values, int64_t n, int32_t n_segments, int32_t k, int64_t *idx,
               void *stream)
{
    clear_error();
    if (!values || !idx)
        return fail(COMET_EINVAL, "comet_topk: NULL pointer");
    if (n < 1 || n_segments < 1 || k < 1 || k > 1024)
        return fail(COMET_EINVAL, "comet_topk: bad sizes (n %lld, segments %d, k %d)",
                    (long long)n, n_segments, k);
    int st = check_device();
    if (st)
        return st;
    ProfScope prof(kProfSelect, (hipStream_t)stream);
    hipLaunchKernelGGL(topk_kernel, dim3(n_segments), dim3(kSelectThreads), 0, (hipStream_t)stream,
                       values, n, k, idx);
    return launched("topk_kernel");
}

int comet_grid_seeds(const double *grids, int32_t n_partitions, const int32_t n[4],
                     const int64_t *idx, int32_t k, double *seeds6, void *stream)
{
    clear_error();
    if (!grids || !n || !idx || !seeds6)
        return fail(COMET_EINVAL, "comet_grid_seeds: NULL pointer");
    if (n_partitions < 1 || k < 1 || (int64_t)n_partitions * k > (1 << 30))
        return fail(COMET_EINVAL, "comet_grid_seeds: bad sizes");
    for (int a = 0; a < 4; ++a)
        if (n[a] < 1)
            return fail(COMET_EINVAL, "comet_grid_seeds: n[%d] < 1", a);
    int st = check_device();
    if (st)
        return st;
    const int64_t total = (int64_t)n_partitions * k;
    hipLaunchKernelGGL(grid_seeds_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, grids, n[0], n[1], n[2], n[3], idx, n_partitions, k,
                       seeds6);
    return launched("grid_seeds_kernel");
}

int comet_batch_variant_count(void) { return kNumBatchVariants; }

int comet_batch_variant_info(int id, int32_t *w, int32_t *nwv, int32_t *chunk, int32_t *blocks,
                             int32_t *direct, int32_t *runs)
{
    if (id < 0 || id >= kNumBatchVariants || !w || !nwv || !chunk)
        return fail(COMET_EINVAL, "comet_batch_variant_info: bad id or NULL pointer");
    *w = kBatchVariants[id].w;
    *nwv = kBatchVariants[id].nwv;
    *chunk = kBatchVariants[id].c;
    if (blocks)
        *blocks = batch_blocks(id);
    if (direct)
        *direct = kBatchVariants[id].direct;
    if (runs)
        *runs = kBatchVariants[id].runs > 0 ? kBatchVariants[id].runs : 1;
    return COMET_OK;
}

int comet_batch_set_variant(int id)
{
    if (id < 0 || id >= kNumBatchVariants)
        return fail(COMET_EINVAL, "comet_batch_set_variant: id %d out of range", id);
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_batch_variant = id;
    return COMET_OK;
}

}  // extern "C"
