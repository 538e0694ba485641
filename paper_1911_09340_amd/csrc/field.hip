// field.hip -- track recording in a magnetic field map (Sec. 2.2.1: each seed's track is
// extrapolated step by step through the solenoid's field map and every step's position
// is recorded for the distance scan). The recorded track has the layout of
// comet_extrapolate_seeds', so comet_dca_rss and comet_select_classify take it as is.
//
// Paper: Yeo, Lee and Kuno, arXiv:1911.09340, Sec. 2.2.1, Alg. 1.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "comet.h"
#include "field_math.h"
#include "host_common.h"

namespace {

using namespace cdev;
using namespace chost;

// One thread per seed: K steps in the map (RK4, or RKN when m.stepper is 1), positions
// stored [3][K + 1][S] with the
// seed index fastest, so the stores of a wave are contiguous; with rho set, the chunk
// radii of the track ([window][S]) are taken while recording.
__global__ __launch_bounds__(256) void rk4_field_record_kernel(const double *__restrict__ seeds,
                                                               int64_t S, FieldMap m,
                                                               double charge, double h, int K,
                                                               double *__restrict__ track,
                                                               double *__restrict__ rho)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S)
        return;
    double x[3] = {seeds[0 * S + s], seeds[1 * S + s], seeds[2 * S + s]};
    double p[3] = {seeds[3 * S + s], seeds[4 * S + s], seeds[5 * S + s]};
    const double p0 = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const double inv = 1.0 / p0;
    const double g = (kKappa * charge) * inv;
    const int64_t P = (int64_t)K + 1;
    double *tx = track + s;
    double *ty = track + P * S + s;
    double *tz = track + 2 * P * S + s;
    ChunkRadius cr;
    double *rs = rho ? rho + s : nullptr;
    const bool rkn = m.stepper == 1;
    const RknConsts kn = rkn_consts(h);
    if (rkn)  // Runge-Kutta-Nystrom carries the unit direction in p
        for (int c = 0; c < 3; ++c)
            p[c] = p[c] * inv;
    CellCache cc;
    auto look = [&](double px, double py, double pz, double (&B)[3]) {
        field_at_cached(m, px, py, pz, B, cc);
    };
    for (int j = 0; j < K; ++j) {
        tx[(int64_t)j * S] = x[0];
        ty[(int64_t)j * S] = x[1];
        tz[(int64_t)j * S] = x[2];
        if (rs)
            cr.add(j, K + 1, x[0], x[1], x[2], rs, S);
        if (rkn)
            rkn_field_step_l(look, kn, g, x, p);
        else
            rk4_field_step_l(look, inv, g, h, x, p);
    }
    tx[(int64_t)K * S] = x[0];
    ty[(int64_t)K * S] = x[1];
    tz[(int64_t)K * S] = x[2];
    if (rs)
        cr.add(K, K + 1, x[0], x[1], x[2], rs, S);
}

}  // namespace

namespace chost {

int launch_field_record(const double *seeds6, int64_t S, const comet_field *field,
                        double charge, double h, int K, double *track, double *rho,
                        hipStream_t stream)
{
    const FieldMap m{field->b, field->nx, field->ny, field->nz, field->x0, field->y0,
                     field->z0, field->dx, field->dy, field->dz, field->stepper};
    const int threads = 256;
    hipLaunchKernelGGL(rk4_field_record_kernel, dim3((unsigned)((S + threads - 1) / threads)),
                       dim3(threads), 0, stream, seeds6, S, m, charge, h, K, track, rho);
    return launched("rk4_field_record_kernel");
}

}  // namespace chost

extern "C" {

int comet_extrapolate_seeds_field(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                                  const comet_field *field, double *track_xyz, void *stream)
{
    clear_error();
    if (!seeds6 || !track_xyz)
        return fail(COMET_EINVAL, "comet_extrapolate_seeds_field: NULL pointer");
    if (n_seeds < 1 || n_seeds > ((int64_t)1 << 40))
        return fail(COMET_EINVAL, "comet_extrapolate_seeds_field: n_seeds = %lld",
                    (long long)n_seeds);
    int st = check_field("comet_extrapolate_seeds_field", field);
    if (st)
        return st;
    st = check_config(cfg);
    if (st)
        return st;
    st = check_device();
    if (st)
        return st;
    ProfScope prof(kProfTrack, (hipStream_t)stream);
    return launch_field_record(seeds6, n_seeds, field, cfg->charge_e, cfg->step_mm,
                               cfg->n_steps, track_xyz, nullptr, (hipStream_t)stream);
}

}  // extern "C"
