// stages.hip -- the stage loop of the event reconstruction (Sec. 3.1): turn partitions
// are scanned one stage at a time from the last turn backwards. After a stage, the hits
// it classified leave the event (later scans see fewer wires), the chosen seed is
// extrapolated backwards to the previous turn's entry for the next stage's
// longitudinal seed (z, p_z), and an event stops when fewer than a minimum of wires
// remain or enough tracks were found.
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 3.1.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "comet.h"
#include "device_math.h"
#include "host_common.h"

namespace {

using namespace cdev;
using namespace chost;

// One thread per seed: the track runs backwards (momentum and charge flipped) with the
// scan's RK4 step; the answer is the first inward crossing of r = radius after an
// outward one, interpolated linearly in r^2 - radius^2 between the step's two states,
// with the momentum flipped back. NaN (and steps = -1) without such a crossing.
__global__ __launch_bounds__(256) void backward_seed_kernel(const double *__restrict__ seeds6,
                                                            int n, double bz, double charge,
                                                            double h, double radius,
                                                            int max_steps,
                                                            double *__restrict__ out6,
                                                            int32_t *__restrict__ steps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double *sd = seeds6 + 6 * (int64_t)i;
    double x = sd[0], y = sd[1], z = sd[2], px = -sd[3], py = -sd[4];
    const double pz = -sd[5];
    const StepConsts kc = step_consts(px, py, pz, bz, -charge, h);
    const double R2 = radius * radius;
    bool out_seen = false;
    double r[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
    int found = -1;
    for (int k = 1; k <= max_steps; ++k) {
        const double ax = x, ay = y, az = z, apx = px, apy = py;
        rk4_step(kc, x, y, z, px, py);
        const double da = (ax * ax + ay * ay) - R2;
        const double db = (x * x + y * y) - R2;
        if (da < 0.0 && db >= 0.0) {
            out_seen = true;
        } else if (out_seen && da >= 0.0 && db < 0.0) {
            const double f = da / (da - db);
            r[0] = fma(f, x - ax, ax);
            r[1] = fma(f, y - ay, ay);
            r[2] = fma(f, z - az, az);
            r[3] = -fma(f, px - apx, apx);
            r[4] = -fma(f, py - apy, apy);
            r[5] = -fma(f, pz - pz, pz);
            found = k;
            break;
        }
    }
    for (int j = 0; j < 6; ++j)
        out6[6 * (int64_t)i + j] = r[j];
    if (steps)
        steps[i] = found;
}

// grids[i] = transverse6[i] with (z, p_z) from ext6[i]; centres (0, |p|, 0, 0).
__global__ __launch_bounds__(256) void stage_grid_kernel(const double *__restrict__ transverse6,
                                                         const double *__restrict__ ext6, int n,
                                                         double h0, double h1, double h2,
                                                         double h3, double *__restrict__ grids)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double *t = transverse6 + 6 * (int64_t)i;
    const double *e = ext6 + 6 * (int64_t)i;
    double *g = grids + 14 * (int64_t)i;
    const double gx = t[0], gy = t[1], gz = e[2], gpx = t[3], gpy = t[4], gpz = e[5];
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
    g[3] = gpx;
    g[4] = gpy;
    g[5] = gpz;
    g[6] = 0.0;
    g[7] = sqrt((gpx * gpx + gpy * gpy) + gpz * gpz);
    g[8] = 0.0;
    g[9] = 0.0;
    g[10] = h0;
    g[11] = h1;
    g[12] = h2;
    g[13] = h3;
}

// The seed's z as a fifth grid axis (Sec. 3.1 gives the seed five degrees of freedom):
// grids[i][u] for u < n_z is stage_grid_kernel's descriptor with the reference z set to
// axis_value(ext z, z_half, n_z, u), the same spacing rule as the other axes.
__global__ __launch_bounds__(256) void stage_grid_z_kernel(const double *__restrict__ transverse6,
                                                           const double *__restrict__ ext6, int n,
                                                           double h0, double h1, double h2,
                                                           double h3, int n_z, double z_half,
                                                           double *__restrict__ grids)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)n * n_z)
        return;
    const int64_t i = q / n_z;
    const int u = (int)(q - i * n_z);
    const double *t = transverse6 + 6 * i;
    const double *e = ext6 + 6 * i;
    double *g = grids + 14 * q;
    const double gx = t[0], gy = t[1], gpx = t[3], gpy = t[4], gpz = e[5];
    g[0] = gx;
    g[1] = gy;
    g[2] = axis_value(e[2], z_half, n_z, u);
    g[3] = gpx;
    g[4] = gpy;
    g[5] = gpz;
    g[6] = 0.0;
    g[7] = sqrt((gpx * gpx + gpy * gpy) + gpz * gpz);
    g[8] = 0.0;
    g[9] = 0.0;
    g[10] = h0;
    g[11] = h1;
    g[12] = h2;
    g[13] = h3;
}

constexpr int kStageThreads = 256;

// Inclusive sum over the block of one int per thread (kStageThreads threads); every
// thread must call it. Returns the inclusive prefix; *total receives the block sum.
__device__ int block_inclusive_sum(int v, int *total)
{
    __shared__ int wsum[kStageThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int s = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(s, off);
        if (lane >= off)
            s += o;
    }
    if (lane == 63)
        wsum[wave] = s;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < kStageThreads / 64; ++w) {
        before += w < wave ? wsum[w] : 0;
        all += wsum[w];
    }
    __syncthreads();  // wsum is reused by the next call
    *total = all;
    return before + s;
}

// Per event (one block): wires that keep at least one hit and the hits kept.
__global__ __launch_bounds__(kStageThreads) void exclude_count_kernel(
    const int32_t *__restrict__ event_wires, const int32_t *__restrict__ wire_offsets,
    const uint8_t *__restrict__ exclude, int32_t *__restrict__ counts)
{
    const int e = blockIdx.x;
    const int w0 = event_wires[e], w1 = event_wires[e + 1];
    int nw = 0, nh = 0;
    for (int i = w0 + threadIdx.x; i < w1; i += kStageThreads) {
        int kept = 0;
        for (int j = wire_offsets[i]; j < wire_offsets[i + 1]; ++j)
            kept += exclude[j] ? 0 : 1;
        nw += kept > 0 ? 1 : 0;
        nh += kept;
    }
    int tw = 0, th = 0;
    (void)block_inclusive_sum(nw, &tw);
    (void)block_inclusive_sum(nh, &th);
    if (threadIdx.x == 0) {
        counts[2 * e] = tw;
        counts[2 * e + 1] = th;
    }
}

// One block: event bases by an exclusive scan over the events, in order.
__global__ __launch_bounds__(kStageThreads) void exclude_scan_kernel(
    const int32_t *__restrict__ counts, int n_events, int32_t *__restrict__ event_wires_out,
    int32_t *__restrict__ hit_base, int32_t *__restrict__ wire_offsets_out)
{
    int wbase = 0, hbase = 0;
    for (int e0 = 0; e0 < n_events; e0 += kStageThreads) {
        const int e = e0 + threadIdx.x;
        const int cw = e < n_events ? counts[2 * e] : 0;
        const int ch = e < n_events ? counts[2 * e + 1] : 0;
        int tw = 0, th = 0;
        const int iw = block_inclusive_sum(cw, &tw);
        const int ih = block_inclusive_sum(ch, &th);
        if (e < n_events) {
            event_wires_out[e] = wbase + iw - cw;
            hit_base[e] = hbase + ih - ch;
        }
        wbase += tw;
        hbase += th;
    }
    if (threadIdx.x == 0) {
        event_wires_out[n_events] = wbase;
        wire_offsets_out[wbase] = hbase;
    }
}

// Per event (one block): the kept wires in order, each with its kept hits in order.
__global__ __launch_bounds__(kStageThreads) void exclude_write_kernel(
    const int32_t *__restrict__ event_wires, const int32_t *__restrict__ wire_offsets,
    const double *__restrict__ drift, const double *__restrict__ wire_ends,
    const int32_t *__restrict__ hit_ids, const uint8_t *__restrict__ exclude,
    const int32_t *__restrict__ event_wires_out, const int32_t *__restrict__ hit_base,
    int32_t *__restrict__ wire_offsets_out, double *__restrict__ drift_out,
    double *__restrict__ wire_ends_out, int32_t *__restrict__ hit_ids_out)
{
    const int e = blockIdx.x;
    const int w0 = event_wires[e], w1 = event_wires[e + 1];
    int wpos = event_wires_out[e], hpos = hit_base[e];
    for (int c0 = w0; c0 < w1; c0 += kStageThreads) {  // block-uniform trip count
        const int i = c0 + threadIdx.x;
        int kept = 0;
        if (i < w1)
            for (int j = wire_offsets[i]; j < wire_offsets[i + 1]; ++j)
                kept += exclude[j] ? 0 : 1;
        const int has = kept > 0 ? 1 : 0;
        int tw = 0, th = 0;
        const int iw = block_inclusive_sum(has, &tw);
        const int ih = block_inclusive_sum(kept, &th);
        if (has) {
            const int wo = wpos + iw - 1;
            int ho = hpos + ih - kept;
            wire_offsets_out[wo] = ho;
            for (int c = 0; c < 6; ++c)
                wire_ends_out[6 * (int64_t)wo + c] = wire_ends[6 * (int64_t)i + c];
            for (int j = wire_offsets[i]; j < wire_offsets[i + 1]; ++j)
                if (!exclude[j]) {
                    drift_out[ho] = drift[j];
                    hit_ids_out[ho] = hit_ids[j];
                    ++ho;
                }
        }
        wpos += tw;
        hpos += th;
    }
}

// Per event (one block): the hits that the stage classified (bit 0 of its mask) get
// the stage number at their original index and are marked for exclusion; events no
// longer active record and exclude nothing.
__global__ __launch_bounds__(kStageThreads) void stage_record_kernel(
    const uint8_t *__restrict__ mask, int64_t mask_stride, const int32_t *__restrict__ event_wires,
    const int32_t *__restrict__ wire_offsets, const int32_t *__restrict__ hit_ids,
    const int32_t *__restrict__ active, int stage, int32_t *__restrict__ stage_of_hit,
    uint8_t *__restrict__ exclude)
{
    const int e = blockIdx.x;
    const int j0 = wire_offsets[event_wires[e]], j1 = wire_offsets[event_wires[e + 1]];
    const bool on = active[e] != 0;
    for (int j = j0 + threadIdx.x; j < j1; j += kStageThreads) {
        const bool cls = on && (mask[(int64_t)e * mask_stride + (j - j0)] & 1);
        exclude[j] = cls ? 1 : 0;
        if (cls)
            stage_of_hit[hit_ids[j]] = stage;
    }
}

// active[e] stays 1 while the stage found a seed, the event has another turn within
// max_stages, and at least min_wires wires remain.
__global__ __launch_bounds__(256) void stage_update_kernel(
    int32_t *__restrict__ active, int n_events, const int64_t *__restrict__ best,
    const int32_t *__restrict__ event_wires_next, const int32_t *__restrict__ n_turns,
    int stage, int max_stages, int min_wires)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_events)
        return;
    const int stages = min(n_turns[e], max_stages);
    const int wires = event_wires_next[e + 1] - event_wires_next[e];
    active[e] = active[e] != 0 && best[e] >= 0 && stage + 1 < stages && wires >= min_wires;
}

// Self-refining of a stage's classified hits (Sec. 3.1), one block per row: the row's
// fitted seed is extrapolated into LDS (thread 0, the RK4 of comet_extrapolate_seeds);
// then one thread per wire of the row's event takes the wire's DCA D to that track,
// keeps a classified hit only while |D - r_j| < lambda, and on a wire left with no
// classified hit classifies the closest hit (first on ties) when its residual is below
// eta. A seed with a NaN component keeps bit 0 of the input mask. Each thread reads
// and writes only its own wire's hits, so mask_out may be mask_in.
constexpr int kRefineThreads = 256;

__global__ __launch_bounds__(kRefineThreads) void self_refine_kernel(
    const double *__restrict__ seeds6, const int32_t *__restrict__ row_event, int n_events,
    double bz, double charge, double h, int K, double lambda, double eta,
    const double *__restrict__ ends, const int32_t *__restrict__ offsets,
    const double *__restrict__ drift, const int32_t *__restrict__ ev_wires,
    const uint8_t *mask_in, uint8_t *mask_out, int64_t mask_stride)
{
    extern __shared__ double pts[];  // [3][K + 1]
    const int r = blockIdx.x;
    const int e = row_event[r];
    if (e < 0 || e >= n_events)
        return;
    const int P = K + 1;
    const int w0 = ev_wires[e], w1 = ev_wires[e + 1];
    const int h0 = offsets[w0];
    const double *sd = seeds6 + 6 * (int64_t)r;
    bool fitted = true;
    for (int c = 0; c < 6; ++c)
        fitted = fitted && !isnan(sd[c]);
    if (fitted && threadIdx.x == 0) {
        double x = sd[0], y = sd[1], z = sd[2], px = sd[3], py = sd[4];
        const StepConsts kc = step_consts(px, py, sd[5], bz, charge, h);
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
    __syncthreads();
    const uint8_t *mi = mask_in + (int64_t)r * mask_stride - h0;
    uint8_t *mout = mask_out + (int64_t)r * mask_stride - h0;
    const int64_t j_end = (int64_t)h0 + mask_stride;  // hits past the row's stride are left alone
    for (int wi = w0 + threadIdx.x; wi < w1; wi += kRefineThreads) {
        const int j0 = offsets[wi];
        const int j1 = (int)min((int64_t)offsets[wi + 1], j_end);
        if (!fitted) {
            for (int j = j0; j < j1; ++j)
                mout[j] = mi[j] & 1;
            continue;
        }
        double f[8];
        wire_frame(ends + 6 * (int64_t)wi, f);
        double qb = INFINITY;
        int kb = 0;
        for (int k = 0; k < P; ++k) {
            double xi, et;
            project(f, pts[k], pts[P + k], pts[2 * P + k], xi, et);
            const double q = fma(xi, xi, et * et);
            if (q < qb) {
                qb = q;
                kb = k;
            }
        }
        const double D = sqrt(refine_dca2(pts, pts + P, pts + 2 * P, 1, P, f, kb, qb));
        int kept = 0;
        for (int j = j0; j < j1; ++j) {
            const bool keep = (mi[j] & 1) && fabs(D - drift[j]) < lambda;
            mout[j] = keep ? 1 : 0;
            kept += keep;
        }
        if (kept == 0) {
            int jb = -1;
            double eb = INFINITY;
            for (int j = j0; j < j1; ++j) {
                const double res = fabs(D - drift[j]);
                if (res < eb) {
                    eb = res;
                    jb = j;
                }
            }
            if (jb >= 0 && eb < eta)
                mout[jb] = 1;
        }
    }
}

}  // namespace

extern "C" {

int comet_backward_seeds(const double *seeds6, int32_t n, const comet_config *cfg, double radius,
                         int32_t max_steps, double *out6, int32_t *steps, void *stream)
{
    clear_error();
    if (!seeds6 || !out6)
        return fail(COMET_EINVAL, "comet_backward_seeds: NULL pointer");
    if (n < 1 || max_steps < 1 || !finite_pos(radius))
        return fail(COMET_EINVAL, "comet_backward_seeds: need n >= 1, max_steps >= 1, radius > 0");
    int st = check_config(cfg);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(backward_seed_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, seeds6, n, cfg->bz_tesla, cfg->charge_e, cfg->step_mm,
                       radius, max_steps, out6, steps);
    return launched("backward_seed_kernel");
}

int comet_stage_grids(const double *transverse6, const double *ext6, int32_t n,
                      const double half[4], double *grids, void *stream)
{
    clear_error();
    if (!transverse6 || !ext6 || !half || !grids)
        return fail(COMET_EINVAL, "comet_stage_grids: NULL pointer");
    if (n < 1)
        return fail(COMET_EINVAL, "comet_stage_grids: n < 1");
    for (int a = 0; a < 4; ++a)
        if (!(half[a] >= 0.0) || !isfinite(half[a]))
            return fail(COMET_EINVAL, "comet_stage_grids: half[%d] must be finite and >= 0", a);
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(stage_grid_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       transverse6, ext6, n, half[0], half[1], half[2], half[3], grids);
    return launched("stage_grid_kernel");
}

int comet_stage_grids_z(const double *transverse6, const double *ext6, int32_t n,
                        const double half[4], int32_t n_z, double z_half, double *grids,
                        void *stream)
{
    clear_error();
    if (!transverse6 || !ext6 || !half || !grids)
        return fail(COMET_EINVAL, "comet_stage_grids_z: NULL pointer");
    if (n < 1 || n_z < 1 || (int64_t)n * n_z > ((int64_t)1 << 31) - 1)
        return fail(COMET_EINVAL, "comet_stage_grids_z: n and n_z must be >= 1");
    for (int a = 0; a < 4; ++a)
        if (!(half[a] >= 0.0) || !isfinite(half[a]))
            return fail(COMET_EINVAL, "comet_stage_grids_z: half[%d] must be finite and >= 0", a);
    if (!(z_half >= 0.0) || !isfinite(z_half))
        return fail(COMET_EINVAL, "comet_stage_grids_z: z_half must be finite and >= 0");
    const int st = check_device();
    if (st)
        return st;
    const int64_t total = (int64_t)n * n_z;
    hipLaunchKernelGGL(stage_grid_z_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, transverse6, ext6, n, half[0], half[1], half[2],
                       half[3], n_z, z_half, grids);
    return launched("stage_grid_z_kernel");
}

size_t comet_exclude_workspace_bytes(int32_t n_events)
{
    if (n_events < 1)
        return 0;
    return align256(sizeof(int32_t) * 3 * (size_t)n_events);
}

int comet_exclude_hits(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                       int32_t n_wires, const double *drift, const double *wire_ends,
                       const int32_t *hit_ids, int32_t n_hits, const uint8_t *exclude,
                       int32_t *event_wires_out, int32_t *wire_offsets_out, double *drift_out,
                       double *wire_ends_out, int32_t *hit_ids_out, void *workspace,
                       size_t workspace_bytes, void *stream)
{
    clear_error();
    if (!event_wires || !wire_offsets || !wire_ends || !hit_ids || !exclude || !event_wires_out ||
        !wire_offsets_out || !wire_ends_out || !hit_ids_out || (n_hits > 0 && (!drift || !drift_out)))
        return fail(COMET_EINVAL, "comet_exclude_hits: NULL pointer");
    if (n_events < 1 || n_wires < 0 || n_hits < 0)
        return fail(COMET_EINVAL, "comet_exclude_hits: bad sizes");
    const size_t need = comet_exclude_workspace_bytes(n_events);
    if (!workspace || workspace_bytes < need)
        return fail(COMET_EWORKSPACE, "comet_exclude_hits: workspace %zu < %zu bytes",
                    workspace_bytes, need);
    const int st = check_device();
    if (st)
        return st;
    hipStream_t hs = (hipStream_t)stream;
    int32_t *counts = (int32_t *)workspace;
    int32_t *hit_base = counts + 2 * (size_t)n_events;
    hipLaunchKernelGGL(exclude_count_kernel, dim3(n_events), dim3(kStageThreads), 0, hs,
                       event_wires, wire_offsets, exclude, counts);
    int s = launched("exclude_count_kernel");
    if (s)
        return s;
    hipLaunchKernelGGL(exclude_scan_kernel, dim3(1), dim3(kStageThreads), 0, hs,
                       (const int32_t *)counts, n_events, event_wires_out, hit_base,
                       wire_offsets_out);
    s = launched("exclude_scan_kernel");
    if (s)
        return s;
    hipLaunchKernelGGL(exclude_write_kernel, dim3(n_events), dim3(kStageThreads), 0, hs,
                       event_wires, wire_offsets, drift, wire_ends, hit_ids, exclude,
                       (const int32_t *)event_wires_out, (const int32_t *)hit_base,
                       wire_offsets_out, drift_out, wire_ends_out, hit_ids_out);
    return launched("exclude_write_kernel");
}

int comet_stage_record(const uint8_t *hit_mask, int64_t mask_stride, int32_t n_events,
                       const int32_t *event_wires, const int32_t *wire_offsets,
                       const int32_t *hit_ids, const int32_t *active, int32_t stage,
                       int32_t *stage_of_hit, uint8_t *exclude, void *stream)
{
    clear_error();
    if (!hit_mask || !event_wires || !wire_offsets || !hit_ids || !active || !stage_of_hit ||
        !exclude)
        return fail(COMET_EINVAL, "comet_stage_record: NULL pointer");
    if (n_events < 1 || mask_stride < 1 || stage < 0)
        return fail(COMET_EINVAL, "comet_stage_record: bad sizes");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(stage_record_kernel, dim3(n_events), dim3(kStageThreads), 0,
                       (hipStream_t)stream, hit_mask, mask_stride, event_wires, wire_offsets,
                       hit_ids, active, stage, stage_of_hit, exclude);
    return launched("stage_record_kernel");
}

int comet_self_refine(const double *seeds6, int32_t n_rows, const int32_t *row_event,
                      const comet_config *cfg, const double *wire_ends, int32_t n_wires,
                      const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                      const int32_t *event_wires, int32_t n_events, double eta,
                      const uint8_t *mask_in, uint8_t *mask_out, int64_t mask_stride,
                      void *stream)
{
    clear_error();
    if (!seeds6 || !row_event || !wire_ends || !wire_offsets || !drift || !event_wires ||
        !mask_in || !mask_out)
        return fail(COMET_EINVAL, "comet_self_refine: NULL pointer");
    if (n_rows < 1 || n_events < 1 || n_wires < 0 || n_hits < 0 || mask_stride < 1)
        return fail(COMET_EINVAL, "comet_self_refine: bad sizes");
    if (!(eta >= 0.0) || !isfinite(eta))
        return fail(COMET_EINVAL, "comet_self_refine: eta must be finite and >= 0");
    int st = check_config(cfg);
    if (st)
        return st;
    if (cfg->n_steps > 2400)
        return fail(COMET_EUNSUPPORTED, "comet_self_refine: n_steps %d > 2400", cfg->n_steps);
    st = check_device();
    if (st)
        return st;
    const size_t lds = sizeof(double) * 3 * (size_t)(cfg->n_steps + 1);
    hipLaunchKernelGGL(self_refine_kernel, dim3(n_rows), dim3(kRefineThreads), lds,
                       (hipStream_t)stream, seeds6, row_event, n_events, cfg->bz_tesla,
                       cfg->charge_e, cfg->step_mm, cfg->n_steps, cfg->lambda_mm, eta, wire_ends,
                       wire_offsets, drift, event_wires, mask_in, mask_out, mask_stride);
    return launched("self_refine_kernel");
}

int comet_stage_update(int32_t *active, int32_t n_events, const int64_t *best,
                       const int32_t *event_wires_next, const int32_t *n_turns, int32_t stage,
                       int32_t max_stages, int32_t min_wires, void *stream)
{
    clear_error();
    if (!active || !best || !event_wires_next || !n_turns)
        return fail(COMET_EINVAL, "comet_stage_update: NULL pointer");
    if (n_events < 1 || stage < 0 || max_stages < 1 || min_wires < 0)
        return fail(COMET_EINVAL, "comet_stage_update: bad sizes");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(stage_update_kernel, dim3((n_events + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, active, n_events, best, event_wires_next, n_turns,
                       stage, max_stages, min_wires);
    return launched("stage_update_kernel");
}

}  // extern "C"
