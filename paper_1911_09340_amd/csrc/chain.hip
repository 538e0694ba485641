// chain.hip -- the pieces of the paper's per-stage chain (Sec. 3.1) that the stage loop
// needs beyond the scans: each stage splits the turn partition's remaining hits into an
// entrance and an exit half, seeds the exit half from where the turn re-enters the seed
// region, scans both halves with several references, vetoes and merges the half sets
// (halves.hip), and takes the best complete set's hits and entrance seed on to the
// self-refining and the backward extrapolation (stages.hip).
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

// One thread per state: from the turn's entry the track runs forwards (the scan's RK4
// step) until it first crosses r = radius inwards after having been outside; the state
// there, interpolated linearly in r^2 - radius^2 between the step's two states, with
// the momentum reversed (the exit half runs back through the turn). NaN and steps = -1
// without such a crossing.
__global__ __launch_bounds__(256) void exit_seed_kernel(const double *__restrict__ states,
                                                        int64_t row_stride, int n, double bz,
                                                        double charge, double h, double radius,
                                                        int max_steps, double *__restrict__ out6,
                                                        int32_t *__restrict__ steps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double *sd = states + row_stride * (int64_t)i;
    double x = sd[0], y = sd[1], z = sd[2], px = sd[3], py = sd[4];
    const double pz = sd[5];
    const StepConsts kc = step_consts(px, py, pz, bz, charge, h);
    const double R2 = radius * radius;
    bool outside = false;
    double r[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
    int found = -1;
    for (int k = 0; k < max_steps; ++k) {
        const double ax = x, ay = y, az = z, apx = px, apy = py;
        rk4_step(kc, x, y, z, px, py);
        const double da = (ax * ax + ay * ay) - R2;
        const double db = (x * x + y * y) - R2;
        outside = outside || da > 0.0;
        if (outside && da >= 0.0 && db < 0.0) {
            const double f = da / (da - db);
            r[0] = fma(f, x - ax, ax);
            r[1] = fma(f, y - ay, ay);
            r[2] = fma(f, z - az, az);
            r[3] = -fma(f, px - apx, apx);
            r[4] = -fma(f, py - apy, apy);
            r[5] = -pz;
            found = k;
            break;
        }
    }
    for (int j = 0; j < 6; ++j)
        out6[6 * (int64_t)i + j] = r[j];
    if (steps)
        steps[i] = found;
}

// Hits of the packed events (the first wire_offsets[event_wires[n_events]] of the
// capacity) split by side: exclude_entrance[j] = 1 for a hit on the exit side,
// exclude_exit[j] = 1 for one on the entrance side; a hit id outside the side table
// leaves both halves.
__global__ __launch_bounds__(256) void half_split_kernel(
    const int32_t *__restrict__ event_wires, int n_events,
    const int32_t *__restrict__ wire_offsets, const int32_t *__restrict__ hit_ids, int n_hits,
    const uint8_t *__restrict__ entrance_side, int n_ids, uint8_t *__restrict__ exclude_entrance,
    uint8_t *__restrict__ exclude_exit)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int used = wire_offsets[event_wires[n_events]];
    if (j >= n_hits || j >= used)
        return;
    const int id = hit_ids[j];
    const bool known = id >= 0 && id < n_ids;
    const bool ent = known && entrance_side[id] != 0;
    exclude_entrance[j] = ent ? 0 : 1;
    exclude_exit[j] = (known && !ent) ? 0 : 1;
}

// wire_layer[w] = hit_layer[hit_ids[first hit of w]] for the packed events' wires (every
// wire of an excluded CSR keeps at least one hit); -1 for an id outside the table.
__global__ __launch_bounds__(256) void wire_layer_kernel(
    const int32_t *__restrict__ event_wires, int n_events,
    const int32_t *__restrict__ wire_offsets, int n_wires, const int32_t *__restrict__ hit_ids,
    const int32_t *__restrict__ hit_layer, int n_ids, int32_t *__restrict__ wire_layer)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_wires || w >= event_wires[n_events])
        return;
    const int j = wire_offsets[w];
    const int id = wire_offsets[w + 1] > j ? hit_ids[j] : -1;
    wire_layer[w] = (id >= 0 && id < n_ids) ? hit_layer[id] : -1;
}

// One wave per event. The chosen pair is the top-ranked complete set (pair[e][0] =
// i F + j: entrance seed i, exit seed j), or (0, 0), the lowest-RSS seed of each side,
// when there is none. The event's hits are walked in order; a hit's rank among the
// event's hits of its own side is its index in that half's mask (the halves keep the
// order), found with a ballot per 64 hits.
__global__ __launch_bounds__(64) void union_halves_kernel(
    const int32_t *__restrict__ pair, const int32_t *__restrict__ n_complete, int F,
    const int32_t *__restrict__ event_wires, const int32_t *__restrict__ wire_offsets,
    const int32_t *__restrict__ hit_ids, const uint8_t *__restrict__ entrance_side, int n_ids,
    const uint8_t *__restrict__ mask_a, int64_t stride_a, const uint8_t *__restrict__ mask_b,
    int64_t stride_b, const double *__restrict__ seeds_a, const int32_t *__restrict__ active,
    uint8_t *__restrict__ mask_out, int64_t stride_out, double *__restrict__ seed_out,
    int64_t *__restrict__ best_out)
{
    const int e = blockIdx.x;
    const int lane = threadIdx.x;
    if (!active[e]) {
        if (lane < 6)
            seed_out[6 * (int64_t)e + lane] = NAN;
        if (lane == 0)
            best_out[e] = -1;
        return;
    }
    const int p0 = n_complete[e] > 0 ? pair[(int64_t)e * F * F] : -1;
    const int i = p0 >= 0 ? p0 / F : 0, j = p0 >= 0 ? p0 % F : 0;
    const double *sa = seeds_a + 6 * ((int64_t)e * F + i);
    if (lane < 6)
        seed_out[6 * (int64_t)e + lane] = sa[lane];
    if (lane == 0)
        best_out[e] = isnan(sa[0]) ? -1 : (int64_t)i * F + j;
    const uint8_t *ma = mask_a + ((int64_t)e * F + i) * stride_a;
    const uint8_t *mb = mask_b + ((int64_t)e * F + j) * stride_b;
    const int h0 = wire_offsets[event_wires[e]], h1 = wire_offsets[event_wires[e + 1]];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int ca = 0, cb = 0;
    for (int base = h0; base < h1; base += 64) {
        const int h = base + lane;
        const bool valid = h < h1;
        int id = valid ? hit_ids[h] : -1;
        const bool known = id >= 0 && id < n_ids;
        const bool ent = valid && known && entrance_side[id] != 0;
        const bool ext = valid && known && entrance_side[id] == 0;
        const uint64_t ba = __ballot(ent), bb = __ballot(ext);
        const int ra = ca + __popcll(ba & below), rb = cb + __popcll(bb & below);
        if (valid && h - h0 < stride_out) {
            uint8_t bit = 0;
            if (ent && ra < stride_a)
                bit = ma[ra] & 1;
            else if (ext && rb < stride_b)
                bit = mb[rb] & 1;
            mask_out[(int64_t)e * stride_out + (h - h0)] = bit;
        }
        ca += __popcll(ba);
        cb += __popcll(bb);
    }
}

}  // namespace

extern "C" {

int comet_exit_seeds(const double *states, int64_t row_stride, int32_t n, const comet_config *cfg,
                     double radius, int32_t max_steps, double *out6, int32_t *steps,
                     void *stream)
{
    clear_error();
    if (!states || !out6)
        return fail(COMET_EINVAL, "comet_exit_seeds: NULL pointer");
    if (n < 1 || row_stride < 6 || max_steps < 1 || !finite_pos(radius))
        return fail(COMET_EINVAL,
                    "comet_exit_seeds: need n >= 1, row_stride >= 6, max_steps >= 1, radius > 0");
    int st = check_config(cfg);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(exit_seed_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       states, row_stride, n, cfg->bz_tesla, cfg->charge_e, cfg->step_mm, radius,
                       max_steps, out6, steps);
    return launched("exit_seed_kernel");
}

int comet_half_split(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                     const int32_t *hit_ids, int32_t n_hits, const uint8_t *entrance_side,
                     int32_t n_ids, uint8_t *exclude_entrance, uint8_t *exclude_exit,
                     void *stream)
{
    clear_error();
    if (!event_wires || !wire_offsets || !hit_ids || !entrance_side || !exclude_entrance ||
        !exclude_exit)
        return fail(COMET_EINVAL, "comet_half_split: NULL pointer");
    if (n_events < 1 || n_hits < 1 || n_ids < 1)
        return fail(COMET_EINVAL, "comet_half_split: bad sizes");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(half_split_kernel, dim3((n_hits + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, event_wires, n_events, wire_offsets, hit_ids, n_hits,
                       entrance_side, n_ids, exclude_entrance, exclude_exit);
    return launched("half_split_kernel");
}

int comet_wire_layers(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                      int32_t n_wires, const int32_t *hit_ids, const int32_t *hit_layer,
                      int32_t n_ids, int32_t *wire_layer, void *stream)
{
    clear_error();
    if (!event_wires || !wire_offsets || !hit_ids || !hit_layer || !wire_layer)
        return fail(COMET_EINVAL, "comet_wire_layers: NULL pointer");
    if (n_events < 1 || n_wires < 1 || n_ids < 1)
        return fail(COMET_EINVAL, "comet_wire_layers: bad sizes");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(wire_layer_kernel, dim3((n_wires + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, event_wires, n_events, wire_offsets, n_wires, hit_ids,
                       hit_layer, n_ids, wire_layer);
    return launched("wire_layer_kernel");
}

int comet_union_halves(const int32_t *pair, const int32_t *n_complete, int32_t n_final,
                       int32_t n_events, const int32_t *event_wires, const int32_t *wire_offsets,
                       const int32_t *hit_ids, const uint8_t *entrance_side, int32_t n_ids,
                       const uint8_t *mask_a, int64_t stride_a, const uint8_t *mask_b,
                       int64_t stride_b, const double *seeds_a, const int32_t *active,
                       uint8_t *mask_out, int64_t stride_out, double *seed_out,
                       int64_t *best_out, void *stream)
{
    clear_error();
    if (!pair || !n_complete || !event_wires || !wire_offsets || !hit_ids || !entrance_side ||
        !mask_a || !mask_b || !seeds_a || !active || !mask_out || !seed_out || !best_out)
        return fail(COMET_EINVAL, "comet_union_halves: NULL pointer");
    if (n_final < 1 || n_final > 64 || n_events < 1 || n_ids < 1 || stride_a < 1 ||
        stride_b < 1 || stride_out < 1)
        return fail(COMET_EINVAL, "comet_union_halves: bad sizes");
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(union_halves_kernel, dim3(n_events), dim3(64), 0, (hipStream_t)stream, pair,
                       n_complete, n_final, event_wires, wire_offsets, hit_ids, entrance_side,
                       n_ids, mask_a, stride_a, mask_b, stride_b, seeds_a, active, mask_out,
                       stride_out, seed_out, best_out);
    return launched("union_halves_kernel");
}

}  // extern "C"
