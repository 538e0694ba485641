// halves.hip -- the half-track step after the seed scans (Sec. 3.1): each turn
// partition is scanned as two half tracks, each ending with its finally selected
// seeds and their half sets of classified hits. A seed whose half set leaves a layer
// without a hit is excluded, and the kept seeds of the two sides are merged
// combinatorially into complete sets.
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 3.1.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "comet.h"
#include "host_common.h"

namespace {

using namespace chost;

constexpr int kVetoThreads = 256;
constexpr int kMaxLayers = 256;
constexpr int kMergeThreads = 1024;
constexpr int kMaxMergeSeeds = 32;  // F^2 pairs, one per thread

// One block per classified seed (row). Every wire of the row's event marks its layer
// when one of its hits has bit 0 set; then thread 0 looks for a gap below the
// outermost marked layer. 1 = vetoed (a gap, or nothing classified), 0 = kept, -1 =
// a wire's layer outside [0, n_layers) or a hit past mask_stride.
__global__ __launch_bounds__(kVetoThreads) void layer_veto_kernel(
    const uint8_t *__restrict__ mask, int64_t mask_stride, const int32_t *__restrict__ row_event,
    const int32_t *__restrict__ event_wires, const int32_t *__restrict__ wire_offsets,
    const int32_t *__restrict__ wire_layer, int n_layers, int32_t *__restrict__ veto)
{
    __shared__ int has[kMaxLayers];
    __shared__ int bad;
    const int64_t row = blockIdx.x;
    for (int l = threadIdx.x; l < n_layers; l += kVetoThreads)
        has[l] = 0;
    if (threadIdx.x == 0)
        bad = 0;
    __syncthreads();
    const int e = row_event[row];
    const int w0 = event_wires[e], w1 = event_wires[e + 1];
    const int h0 = wire_offsets[w0];
    const uint8_t *m = mask + row * mask_stride;
    for (int i = w0 + threadIdx.x; i < w1; i += kVetoThreads) {
        const int L = wire_layer[i];
        const int j1 = wire_offsets[i + 1];
        if (L < 0 || L >= n_layers || j1 - h0 > mask_stride) {
            atomicOr(&bad, 1);
            continue;
        }
        int any = 0;
        for (int j = wire_offsets[i]; j < j1; ++j)
            any |= m[j - h0] & 1;
        if (any)
            atomicOr(&has[L], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int v;
        if (bad) {
            v = -1;
        } else {
            int outer = -1;
            for (int l = 0; l < n_layers; ++l)
                if (has[l])
                    outer = l;
            v = outer < 0 ? 1 : 0;
            for (int l = 0; l <= outer; ++l)
                if (!has[l])
                    v = 1;
        }
        veto[row] = v;
    }
}

// One block per partition, one thread per pair k = i F + j. A pair is a complete set
// when neither seed is vetoed and neither RSS is NaN; its rank is the number of
// complete sets before it in (combined RSS, k) order, so every rank is written once.
__global__ __launch_bounds__(kMergeThreads) void merge_halves_kernel(
    const double *__restrict__ rss_a, const int32_t *__restrict__ veto_a,
    const double *__restrict__ rss_b, const int32_t *__restrict__ veto_b, int F,
    int32_t *__restrict__ pair, double *__restrict__ pair_rss, int32_t *__restrict__ n_complete)
{
    __shared__ double sv[kMergeThreads];
    __shared__ int ok[kMergeThreads];
    const int64_t p = blockIdx.x;
    const int FF = F * F;
    const int k = threadIdx.x;
    double v = 0.0;
    int valid = 0;
    if (k < FF) {
        const int i = k / F, j = k % F;
        const double a = rss_a[p * F + i], b = rss_b[p * F + j];
        valid = veto_a[p * F + i] == 0 && veto_b[p * F + j] == 0 && !isnan(a) && !isnan(b);
        v = a + b;
    }
    sv[k] = v;
    ok[k] = valid;
    const int n_valid = __syncthreads_count(valid);
    if (valid) {
        int rank = 0;
        for (int m = 0; m < FF; ++m)
            rank += ok[m] && (sv[m] < v || (sv[m] == v && m < k));
        pair[p * FF + rank] = k;
        pair_rss[p * FF + rank] = v;
    }
    if (k >= n_valid && k < FF) {
        pair[p * FF + k] = -1;
        pair_rss[p * FF + k] = NAN;
    }
    if (k == 0 && n_complete)
        n_complete[p] = n_valid;
}

}  // namespace

extern "C" {

int comet_layer_veto(const uint8_t *hit_mask, int64_t mask_stride, int32_t n_rows,
                     const int32_t *row_event, const int32_t *event_wires, int32_t n_events,
                     const int32_t *wire_offsets, const int32_t *wire_layer, int32_t n_wires,
                     int32_t n_layers, int32_t *veto, void *stream)
{
    clear_error();
    if (!hit_mask || !row_event || !event_wires || !wire_offsets || !wire_layer || !veto)
        return fail(COMET_EINVAL, "comet_layer_veto: NULL pointer");
    if (n_rows < 1 || n_events < 1 || n_wires < 0 || mask_stride < 1)
        return fail(COMET_EINVAL, "comet_layer_veto: bad sizes");
    if (n_layers < 1 || n_layers > kMaxLayers)
        return fail(COMET_EINVAL, "comet_layer_veto: n_layers must be 1..%d", kMaxLayers);
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(layer_veto_kernel, dim3(n_rows), dim3(kVetoThreads), 0,
                       (hipStream_t)stream, hit_mask, mask_stride, row_event, event_wires,
                       wire_offsets, wire_layer, n_layers, veto);
    return launched("layer_veto_kernel");
}

int comet_merge_halves(const double *rss_a, const int32_t *veto_a, const double *rss_b,
                       const int32_t *veto_b, int32_t n_partitions, int32_t n_seeds,
                       int32_t *pair, double *pair_rss, int32_t *n_complete, void *stream)
{
    clear_error();
    if (!rss_a || !veto_a || !rss_b || !veto_b || !pair || !pair_rss)
        return fail(COMET_EINVAL, "comet_merge_halves: NULL pointer");
    if (n_partitions < 1 || n_seeds < 1 || n_seeds > kMaxMergeSeeds)
        return fail(COMET_EINVAL, "comet_merge_halves: need n_partitions >= 1 and 1 <= n_seeds <= %d",
                    kMaxMergeSeeds);
    const int st = check_device();
    if (st)
        return st;
    hipLaunchKernelGGL(merge_halves_kernel, dim3(n_partitions), dim3(kMergeThreads), 0,
                       (hipStream_t)stream, rss_a, veto_a, rss_b, veto_b, n_seeds, pair, pair_rss,
                       n_complete);
    return launched("merge_halves_kernel");
}

}  // extern "C"
