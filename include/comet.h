/*
 * comet.h -- C ABI of the MI355X (gfx950) seed-scan library.
 *
 * The operations are those of Yeo, Lee and Kuno, "GPU-accelerated event
 * reconstruction for the COMET Phase-I experiment" (arXiv:1911.09340): seeds on a
 * grid over prior ranges (Sec. 2.1, Sec. 3.1) are extrapolated into recorded tracks
 * (Sec. 2.2.1, Alg. 1); every wire's distance of closest approach to each track
 * (Sec. 2.2.2, Alg. 2) gives the residual sum of squares of Eq. 1; the lowest-RSS
 * seed is chosen, re-scanned on a finer grid around it, and the hits whose residual
 * is below the cutoff are classified to it (Sec. 2.1).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (memory of the current HIP device) unless
 *     marked "host". The caller owns all memory; the library never allocates,
 *     frees or synchronises in these calls.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls
 *     are asynchronous on it; a fault inside a kernel surfaces at the caller's
 *     next synchronisation, not in the return code.
 *   - Return 0 (COMET_OK) or a negative status; comet_status_string() explains it,
 *     comet_last_error() gives details of the last failure on the calling thread.
 *     Argument checks cover what is visible on the host (NULL pointers, sizes,
 *     configuration values); the contents of device arrays are not inspected.
 *   - Units: mm, MeV/c, tesla, charge in units of e.
 *   - Floating point is IEEE binary64 throughout, evaluated in a fixed order
 *     without contraction, so results are deterministic run to run.
 *   - Only gfx950 devices are supported (COMET_EUNSUPPORTED otherwise).
 */
#ifndef COMET_H
#define COMET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum comet_status {
    COMET_OK = 0,
    COMET_EINVAL = -1,      /* invalid argument (NULL pointer, bad size or value) */
    COMET_EWORKSPACE = -2,  /* workspace NULL or smaller than required */
    COMET_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
    COMET_EUNSUPPORTED = -4 /* current device is not gfx950, or an unsupported option */
};

/* Host struct. Track stepping and Eq. 1 settings.
 *   bz_tesla  uniform axial field B_z (finite)
 *   charge_e  particle charge in e (finite; electron = -1)
 *   step_mm   RK4 path-length step h (> 0, finite)
 *   n_steps   K >= 1; a recorded track has K + 1 points
 *   lambda_mm cutoff lambda of Eq. 1 and of the classification (> 0, finite) */
typedef struct comet_config {
    double bz_tesla;
    double charge_e;
    double step_mm;
    int32_t n_steps;
    int32_t reserved; /* must be 0 */
    double lambda_mm;
} comet_config;

/* Seed grid (Sec. 2.1: a grid search over the prior range of each seed component;
 * Sec. 3.1: the seed set combines the grids of the components).
 *   grid   device double[14]: reference state (x, y, z, px, py, pz), axis centres
 *          (arc offset along the circle of the reference radius [mm], |p| [MeV/c],
 *          polar-angle offset [rad], azimuth offset [rad]), axis half-spans (same units)
 *   n      host int32[4]: points per axis (each >= 1); axis 3 runs fastest
 *   seeds6 device double[6][n_seeds] (SoA: x, y, z, px, py, pz), written
 *   n_seeds must equal n[0] n[1] n[2] n[3]
 * Axis value i is centre + half (2i - (n-1)) / (n-1) (the centre when n = 1); an
 * offset v rotates by 2 atan(tau) with tau = v / (2 r0) for the arc offset (r0 =
 * transverse radius of the reference point) and tau = v / 2 for the angles.
 * The reference momentum must have a non-zero transverse part. */
int comet_seed_grid(const double *grid, const int32_t n[4], double *seeds6, int64_t n_seeds,
                    void *stream);

/* Finer re-scan around the chosen seed (Sec. 2.1): for each axis with n > 1 the
 * centre moves to the value at the chosen seed's index and the half-span becomes
 * one spacing of the previous grid, 2 half / (n - 1).
 *   grid  device double[14], updated in place
 *   n     host int32[4], the grid's points per axis
 *   best  device int64[1]: chosen seed index of the current grid (< 0: no change) */
int comet_refine_grid(double *grid, const int32_t n[4], const int64_t *best, void *stream);

/* Track recording (Sec. 2.2.1, Alg. 1): each seed is stepped with fixed-step
 * classical RK4 in path length through the uniform field (|p| constant) and every
 * position is recorded.
 *   seeds6    device double[6][n_seeds] (SoA)
 *   cfg       host; uses bz_tesla, charge_e, step_mm, n_steps
 *   track_xyz device double[3][n_steps + 1][n_seeds], written: coordinate-major,
 *             then step, then seed (consecutive seeds are adjacent in memory) */
int comet_extrapolate_seeds(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                            double *track_xyz, void *stream);

/* Track recording in a field map (Sec. 2.2.1 extrapolates through the solenoid's
 * field map). The map is B (tesla) on a regular grid: b device double[nz][ny][nx][3]
 * at nodes (x0 + i dx, y0 + j dy, z0 + k dz) mm; B at a point is the trilinear
 * interpolation of its cell (each coordinate clamped to the grid). The ODE is
 * dx/ds = p / |p_seed|, dp/ds = (kappa q / |p_seed|) (p x B(x)), stepped with
 * classical RK4 (every stage reads B at its own position), step cfg->step_mm,
 * cfg->n_steps steps; cfg->bz_tesla is not used. The output is as for
 * comet_extrapolate_seeds, so comet_dca_rss and comet_select_classify take it
 * unchanged. nx, ny, nz >= 2, spacings > 0. The caller owns the map.
 * stepper 1 selects Runge-Kutta-Nystrom instead (the paper's extrapolation): Nystrom's
 * fourth-order method for x'' = g (x' x B(x)) in the unit direction t = x' (t = p / |p|
 * at the seed), a(x, t) = g (t x B): a1 = a(x, t); xm = (x + h/2 t) + h^2/8 a1;
 * a2 = a(xm, t + h/2 a1); a3 = a(xm, t + h/2 a2); xe = (x + h t) + h^2/2 a3;
 * a4 = a(xe, t + h a3); x <- (x + h t) + h^2/6 ((a1 + a2) + a3);
 * t <- t + h/6 (((a1 + 2 a2) + 2 a3) + a4): three reads of the map per step. Every
 * call that takes a comet_field honours it. */
typedef struct comet_field {
    const double *b;
    int32_t nx, ny, nz;
    int32_t stepper; /* 0: classical RK4; 1: Runge-Kutta-Nystrom */
    double x0, y0, z0;
    double dx, dy, dz;
} comet_field;
int comet_extrapolate_seeds_field(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                                  const comet_field *field, double *track_xyz, void *stream);

/* Bytes of workspace comet_dca_rss needs for n_seeds seeds of n_points recorded points
 * and n_wires wires (0 for invalid sizes). */
size_t comet_dca_workspace_bytes(int64_t n_seeds, int32_t n_points, int32_t n_wires);

/* Distance of closest approach and Eq. 1 (Sec. 2.1, Sec. 2.2.2, Alg. 2).
 * For every seed and wire: the recorded point closest to the wire line (first
 * index on ties) is refined over its two adjacent chords to the DCA D; the wire
 * contributes d^2 with d = min(lambda, min_j |D - r_j|) over its hits j (lambda for
 * a wire without hits); rss[s] is the sum over wires in wire order. The scan skips
 * runs of points that a distance bound proves cannot hold or tie a wire's closest
 * point (the radii of 16-point windows of each track go to the workspace first); the
 * results are those of the full scan for any track.
 *   track_xyz    device double[3][n_points][n_seeds] from comet_extrapolate_seeds
 *   n_points     must equal cfg->n_steps + 1
 *   wire_ends    device double[n_wires][6]: both endpoints of each wire (the wire is
 *                the infinite line through them; they must differ)
 *   wire_offsets device int32[n_wires + 1]: CSR, hits of wire i are
 *                [wire_offsets[i], wire_offsets[i+1]); wire_offsets[0] = 0,
 *                non-decreasing, wire_offsets[n_wires] = n_hits
 *   drift        device double[n_hits]: drift distances r_j (finite)
 *   rss          device double[n_seeds], written
 *   workspace    device, >= comet_dca_workspace_bytes(n_seeds, n_points, n_wires) bytes,
 *                256-byte aligned; contents on entry are ignored */
int comet_dca_rss(const double *track_xyz, int64_t n_seeds, int32_t n_points,
                  const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                  const double *drift, int32_t n_hits, const comet_config *cfg, double *rss,
                  void *workspace, size_t workspace_bytes, void *stream);

/* comet_extrapolate_seeds (field == NULL) or comet_extrapolate_seeds_field (field set)
 * followed by comet_dca_rss, in one call (Alg. 1 then Alg. 2 and Eq. 1): the track is
 * written to track_xyz as there, and the radii of its 16-point windows, which the
 * distance bound needs, are taken while it is recorded instead of by a second read of
 * the track. rss and the track are those of the separate calls, bit for bit.
 * Arguments as in those calls; n_points is cfg->n_steps + 1. */
int comet_track_dca_rss(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                        const comet_field *field, const double *wire_ends, int32_t n_wires,
                        const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                        double *track_xyz, double *rss, void *workspace, size_t workspace_bytes,
                        void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): comet_track_dca_rss with the
 * workspace taken from a fixed array in device memory instead of an argument.
 * comet_static_scratch_bytes() is that array's size (64 MiB); each GPU the library
 * runs on holds its own copy until the process ends, and its address on a device is
 * looked up on the first call made with that device current. The call allocates and
 * frees nothing and does not time its launches (comet_profile_begin does not see it).
 * It returns COMET_EWORKSPACE, before any device work, when
 * comet_dca_workspace_bytes(n_seeds, cfg->n_steps + 1, n_wires) exceeds the array (split
 * the seeds into smaller calls). Every call on one GPU uses the same array, so calls
 * that overlap on one GPU (different streams or threads) race and give wrong results;
 * the array needs no clearing between calls (every byte a call reads it writes first).
 * Arguments otherwise as comet_track_dca_rss. */
size_t comet_static_scratch_bytes(void);
int comet_track_dca_rss_static(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                               const comet_field *field, const double *wire_ends,
                               int32_t n_wires, const int32_t *wire_offsets, const double *drift,
                               int32_t n_hits, double *track_xyz, double *rss, void *stream);

/* Seed selection and hit classification (Sec. 2.1).
 * best[0] = index of the lowest rss (ties: lowest index; NaN never chosen; -1 if
 * every value is NaN). When hit_mask is not NULL the chosen seed's track is read
 * from track_xyz, D is recomputed for every wire, and on each wire the hit with
 * the smallest |D - r_j| (lowest index on ties) gets bit 0 of hit_mask when that
 * residual is below lambda (strictly) and bit 1 when it lies within 1e-9 mm of
 * lambda (borderline); all other hits get 0.
 *   top_k        1..1024: best[0..top_k) receives the top_k smallest RSS in increasing
 *                order (ties: lower index; -1 past the last non-NaN value); the hits
 *                are classified for best[0]
 *   best         device int64[top_k], written
 *   hit_mask     device uint8[n_hits] or NULL (selection only)
 *   n_borderline device int32[1] or NULL: number of borderline hits
 *   dca_best     device double[n_wires] or NULL: D of each wire for the chosen seed
 * The track and wire arguments are as in comet_dca_rss (ignored when hit_mask,
 * n_borderline and dca_best are all NULL). */
int comet_select_classify(const double *rss, int64_t n_seeds, const double *track_xyz,
                          int32_t n_points, const double *wire_ends, int32_t n_wires,
                          const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                          const comet_config *cfg, int32_t top_k, int64_t *best,
                          uint8_t *hit_mask, int32_t *n_borderline, double *dca_best,
                          void *stream);

/* ------------------------------------------------------------ derivatives
 * Eq. 1's RSS is not smooth (Sec. 2.1), but it is smooth piecewise: with each wire's
 * closest recorded point, winning chord and closest hit fixed, D_i and the capped
 * residuals are differentiable in the six seed components (x, y, z, px, py, pz).
 *
 * comet_rss_adjoint: for every seed, the track is recomputed (the same RK4 steps as
 * comet_extrapolate_seeds, so every D_i and choice equals the forward path's; the
 * closest point is searched with a distance bound that keeps the first index of the
 * minimum). The derivatives of the recorded points come in closed form: in a uniform
 * field the RK4 step is linear in the transverse momentum (a complex factor per
 * step), so point k is the seed plus a geometric sum of k such factors, taken by
 * binary powering. A wire is active when its closest hit's residual e_i = D_i - r_j
 * satisfies |e_i| < lambda; its row is J_i = dD_i/d(seed).
 *   seeds6       device double[6][n_seeds] (SoA)
 *   cfg          host; n_steps <= 2400
 *   wire_ends, wire_offsets, drift: as in comet_dca_rss
 *   event_wires  device int32[E+1] or NULL; seed_event device int32[n_seeds] or NULL
 *                (both or neither): seed s uses the wires
 *                [event_wires[seed_event[s]], event_wires[seed_event[s]+1]); with
 *                NULL every seed uses all wires
 * Outputs (device, each may be NULL):
 *   rss   double[n_seeds]: Eq. 1, summed in wire order (bit for bit the forward
 *         path's RSS, comet_dca_rss)
 *   grad  double[n_seeds][6]: d rss / d seed = sum over active wires of 2 e_i J_i
 *   jtj   double[n_seeds][21]: sum over active wires of J_i J_i^T, packed upper
 *         triangle, row-major ((0,0), (0,1), ..., (0,5), (1,1), ...)
 *   jte   double[n_seeds][6]: sum over active wires of J_i e_i
 *   dca, resid  double[n_seeds][n_wires]: D_i and e_i (NaN for a wire without hits)
 *   jac   double[n_seeds][n_wires][6]: J_i for active wires, 0 for capped ones
 * Per-wire outputs are written only for the seed's own event's wires. */
int comet_rss_adjoint(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                      const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                      const double *drift, int32_t n_hits, const int32_t *event_wires,
                      const int32_t *seed_event, double *rss, double *grad, double *jtj,
                      double *jte, double *dca, double *resid, double *jac, void *stream);

/* Bytes of workspace comet_lm_refine (and comet_lm_refine_field) needs for n_seeds
 * seeds with tracks of n_steps RK4 steps (0 if n_seeds < 1 or n_steps is outside
 * 1..2400). In a uniform field the refinement records every evaluation's tracks, one
 * seed per lane, into the workspace (24 (n_steps + 1) bytes per seed) before the
 * adjoint blocks load them. */
size_t comet_lm_workspace_bytes(int64_t n_seeds, int32_t n_steps);

/* Levenberg-Marquardt refinement of every seed in place, on the device, with a
 * fixed number of iterations (no host synchronisation, so it can be captured in a
 * HIP graph). Each iteration solves (A + mu diag(A)) delta = -b by Cholesky, where A
 * and b are comet_rss_adjoint's jtj and jte at the current seed, evaluates the trial
 * seed, and accepts it when its RSS is lower (mu <- mu / 10), otherwise keeps the seed
 * (mu <- 10 mu); a matrix that is not positive definite counts as a rejection.
 *   seeds6     device double[6][n_seeds], updated
 *   n_iter     0..1000 iterations; mu0 > 0 initial damping
 *   rss        device double[n_seeds]: RSS at the final seeds
 *   n_accepted device int32[n_seeds] or NULL: accepted steps per seed
 *   workspace  device, >= comet_lm_workspace_bytes(n_seeds, cfg->n_steps), 256-byte
 *              aligned
 * Other arguments as in comet_rss_adjoint. */
int comet_lm_refine(double *seeds6, int64_t n_seeds, const comet_config *cfg,
                    const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                    const double *drift, int32_t n_hits, const int32_t *event_wires,
                    const int32_t *seed_event, int32_t n_iter, double mu0, double *rss,
                    int32_t *n_accepted, void *workspace, size_t workspace_bytes,
                    void *stream);

/* Derivatives and Levenberg-Marquardt in a field map (Sec. 2.2.1: the tracks run
 * through the solenoid's map, as comet_extrapolate_seeds_field records them).
 *
 * comet_rss_jacobian_field: the outputs of comet_rss_adjoint (same layouts, same
 * active-wire rule, rss in the same tree order) for tracks in the map `field` (host
 * struct, as in comet_extrapolate_seeds_field; cfg->bz_tesla is not used). The
 * derivatives are taken in forward mode: six tangents of the RK4 state, one per seed
 * component, are carried along the steps, with dB/dx of the trilinear interpolation
 * (zero along a coordinate clamped to the grid), and J_i = n_i . dP/d(seed) at the
 * wire's closest chord point. One block per seed; an event may hold at most 1024
 * wires: a seed of a larger event gets NaN rss, grad, jtj and jte and no per-wire
 * outputs. cfg->n_steps <= 2400.
 *
 * comet_lm_refine_field: comet_lm_refine with these derivatives and RSS (tracks in the
 * map); arguments, workspace and iteration rule as there. */
int comet_rss_jacobian_field(const double *seeds6, int64_t n_seeds, const comet_config *cfg,
                             const comet_field *field, const double *wire_ends, int32_t n_wires,
                             const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                             const int32_t *event_wires, const int32_t *seed_event, double *rss,
                             double *grad, double *jtj, double *jte, double *dca, double *resid,
                             double *jac, void *stream);
int comet_lm_refine_field(double *seeds6, int64_t n_seeds, const comet_config *cfg,
                          const comet_field *field, const double *wire_ends, int32_t n_wires,
                          const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                          const int32_t *event_wires, const int32_t *seed_event, int32_t n_iter,
                          double mu0, double *rss, int32_t *n_accepted, void *workspace,
                          size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ batches of events
 * The whole Sec. 2.1 path (grid scan, argmin, n_refine finer re-scans, classification)
 * for every turn partition of many events with uneven wire, hit and turn counts.
 * Events are packed in one CSR: event e owns wires [event_wires[e], event_wires[e+1]),
 * wire i owns hits [wire_offsets[i], wire_offsets[i+1]). Partition p belongs to
 * event part_event[p] and starts from the grid descriptor grids[p] (layout as in
 * comet_seed_grid; every partition uses the same n, so S = n0 n1 n2 n3 seeds).
 *
 * Each scan is one persistent launch: blocks take work items (a partition and a run
 * of consecutive 64-seed tiles) from an atomic counter, build the seeds from the
 * descriptor, record their RK4 tracks into per-block scratch (no track array in HBM)
 * and scan the partition's event wires; per-seed RSS are summed in wire order and
 * equal those of
 * comet_dca_rss bit for bit. A per-partition completion counter lets the block that
 * finishes a partition's last tile select its best seed inside the same launch. The
 * calls on `stream` are: a wire-frame kernel, then per scan [refine (not before the
 * first), counter reset, persistent scan], then classification (skipped when
 * best_seed, best_rss, hit_mask and n_borderline are all NULL). No host
 * synchronisation and no allocation: capturable.
 *   wire_ends, wire_offsets, drift   packed events, device (n_wires >= 1)
 *   event_wires  device int32[n_events + 1]; part_event device int32[n_partitions]
 *   grids_init   device double[n_partitions][14] or NULL: copied into grids first (by
 *                a kernel), so that a replayed graph starts from the same grids
 *   grids        device double[n_partitions][14], updated by the re-scans
 *   n            host int32[4]; cfg host (n_steps <= 2400); n_refine 0..100
 *   rss          device double[n_partitions][S]: the last scan's RSS
 *   best         device int64[n_partitions]: argmin in the last grid (-1: all NaN)
 *   best_seed    device double[n_partitions][6] or NULL: the chosen seed (NaN if none)
 *   best_rss     device double[n_partitions] or NULL
 *   hit_mask     device uint8[n_partitions][mask_stride] or NULL: bits as in
 *                comet_select_classify for the partition's event hits, indexed by
 *                hit - wire_offsets[event_wires[e]]; mask_stride >= the most hits of an
 *                event
 *   n_borderline device int32[n_partitions] or NULL
 *   max_items    > 0: scan only the first max_items 64-seed tiles (partition-major) of
 *                every scan (for timing shapes; the other RSS are not written, and a
 *                partition not scanned in full keeps best = -1). A tile is 64
 *                consecutive seeds, or for the blocked shapes a 2 x 2 x 4 x 4 block of the
 *                grid when its axes allow one.
 *   workspace    >= comet_batch_workspace_bytes(n_wires, n_steps, n_partitions),
 *                256-byte aligned */
size_t comet_batch_workspace_bytes(int32_t n_wires, int32_t n_steps, int32_t n_partitions);
int comet_batch_scan(const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                     const double *drift, int32_t n_hits, const int32_t *event_wires,
                     int32_t n_events, const int32_t *part_event, int32_t n_partitions,
                     const double *grids_init, double *grids, const int32_t n[4],
                     const comet_config *cfg, int32_t n_refine, double *rss, int64_t *best,
                     double *best_seed, double *best_rss, uint8_t *hit_mask,
                     int64_t mask_stride, int32_t *n_borderline, int64_t max_items,
                     void *workspace, size_t workspace_bytes, void *stream);

/* comet_batch_scan over the partitions of the events with event_active[e] != 0 only
 * (device int32[n_events]; the stage loop of Sec. 3.1 passes the events still being
 * reconstructed): the work items of the other partitions are skipped, so their rss is
 * not written and their best stays -1 (and their hits get mask 0). Other arguments as
 * comet_batch_scan (max_items is 0). */
int comet_batch_scan_active(const double *wire_ends, int32_t n_wires,
                            const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                            const int32_t *event_wires, int32_t n_events,
                            const int32_t *part_event, int32_t n_partitions,
                            const double *grids_init, double *grids, const int32_t n[4],
                            const comet_config *cfg, int32_t n_refine, double *rss,
                            int64_t *best, double *best_seed, double *best_rss,
                            uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                            const int32_t *event_active, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Several reference seeds per partition (Sec. 2.1 selects several low-RSS seeds as
 * references for the next scan). comet_topk: for each of n_segments rows of n values,
 * idx[row][0..k) = the k smallest values' indices in increasing order (ties: lower
 * index; NaN never chosen; -1 past the last non-NaN value); k 1..1024.
 * comet_grid_seeds: seeds6[:, p k + r] = seed idx[p k + r] of grids[p] (NaN for -1),
 * seeds6 device double[6][n_partitions k]. */
int comet_topk(const double *values, int64_t n, int32_t n_segments, int32_t k, int64_t *idx,
               void *stream);
int comet_grid_seeds(const double *grids, int32_t n_partitions, const int32_t n[4],
                     const int64_t *idx, int32_t k, double *seeds6, void *stream);

/* Sparse reference seeds (Sec. 2.1: several low-RSS seeds, far enough apart that the
 * finer seed sets fetched around them do not overlap, seed the next scan). Group g
 * has n_sub grids grids[g][u][14] (same n for all, S = n0 n1 n2 n3) and their RSS
 * rss[g][u][S]; candidate j = u S + i is seed i of grid u. A candidate's box has the
 * centre of its axis values and, per axis, the refined half-span 2 half / (n - 1) (the
 * grid's centre and half-span where n = 1). Two boxes overlap when on every axis the
 * centres are equal or differ by less than 0.999999999 (h1 + h2). Greedy in increasing
 * (rss, j): a candidate is taken when its box overlaps none taken before; NaN is never
 * taken. For the r-th reference of group g (output row g n_ref + r):
 *   ref_idx    device int64[n_groups][n_ref]: j (-1 past the last one taken)
 *   ref_rss    device double[n_groups][n_ref] or NULL: its RSS (NaN past the last)
 *   new_grids  device double[n_groups][n_ref][14]: grid u refined around seed i (as
 *              comet_refine_grid); past the last taken, a copy of reference 0's (of
 *              grids[g][0] when none was taken)
 *   ref_grids  device double[n_groups][n_ref][14] or NULL: grid u itself (same filling)
 *   ref_local  device int64[n_groups][n_ref] or NULL: i = j mod S (-1 past the last)
 * n_ref 1..64, n_sub S < 2^31. One block per group, on `stream`; no allocation. */
int comet_sparse_select(const double *grids, const double *rss, int32_t n_groups, int32_t n_sub,
                        const int32_t n[4], int32_t n_ref, int64_t *ref_idx, double *ref_rss,
                        double *new_grids, double *ref_grids, int64_t *ref_local, void *stream);

/* comet_batch_scan with every track recorded in the field map `field` (host struct as in
 * comet_extrapolate_seeds_field; RK4 or RKN by its stepper; cfg->bz_tesla is not used),
 * in the persistent kernel as there (one fixed kernel shape: W = 4, 8 waves, 16-point
 * chunks, every wave on its own), and the classification with the map's track. */
int comet_batch_scan_field(const double *wire_ends, int32_t n_wires,
                           const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                           const int32_t *event_wires, int32_t n_events,
                           const int32_t *part_event, int32_t n_partitions,
                           const double *grids_init, double *grids, const int32_t n[4],
                           const comet_config *cfg, const comet_field *field, int32_t n_refine,
                           double *rss, int64_t *best, double *best_seed, double *best_rss,
                           uint8_t *hit_mask, int64_t mask_stride, int32_t *n_borderline,
                           int64_t max_items, void *workspace, size_t workspace_bytes,
                           void *stream);

/* The classification step of comet_batch_scan on its own (Sec. 2.1, hit classification
 * of the chosen seed): for partition p, seed best[p] of grids[p] (best[p] < 0: NaN seed,
 * empty mask) is extrapolated and its hits classified as comet_select_classify does.
 * Arguments as in comet_batch_scan; rss (device double[n_partitions][S]) may be NULL
 * only when best_rss is NULL. Launches one kernel on `stream`. */
int comet_batch_classify(const double *grids, int32_t n_partitions, const int32_t n[4],
                         const int64_t *best, const double *rss, const double *wire_ends,
                         int32_t n_wires, const int32_t *wire_offsets, const double *drift,
                         int32_t n_hits, const int32_t *event_wires, int32_t n_events,
                         const int32_t *part_event, const comet_config *cfg, double *best_seed,
                         double *best_rss, uint8_t *hit_mask, int64_t mask_stride,
                         int32_t *n_borderline, void *stream);
/* The same with the chosen seed's track in the field map `field`. */
int comet_batch_classify_field(const double *grids, int32_t n_partitions, const int32_t n[4],
                               const int64_t *best, const double *rss, const double *wire_ends,
                               int32_t n_wires, const int32_t *wire_offsets,
                               const double *drift, int32_t n_hits, const int32_t *event_wires,
                               int32_t n_events, const int32_t *part_event,
                               const comet_config *cfg, const comet_field *field,
                               double *best_seed, double *best_rss, uint8_t *hit_mask,
                               int64_t mask_stride, int32_t *n_borderline, void *stream);

/* Half tracks (Sec. 3.1): a turn partition is scanned as two half tracks, entrance and
 * exit, each with its own hits; each side ends with its finally selected seeds and
 * their half sets of classified hits.
 *
 * comet_layer_veto: a seed whose half set leaves a layer without a hit is excluded.
 * Row r is one classified seed of packed event row_event[r] (event CSR as in
 * comet_batch_scan; hit_mask[r] indexed by hit - wire_offsets[event_wires[e]], bit 0 =
 * classified). Its half track runs from in front of the first layer out to its
 * outermost classified layer L, so layers 0..L must each hold a classified hit.
 *   veto   device int32[n_rows]: 1 vetoed (a layer missing, or nothing classified),
 *          0 kept, -1 invalid row (a wire_layer outside [0, n_layers) or a hit index
 *          past mask_stride)
 *   wire_layer  device int32[n_wires]; n_layers 1..256. One block per row.
 *
 * comet_merge_halves: complete sets are formed by merging one half set of each side.
 * For partition p, entrance seed i and exit seed j (n_seeds = F each, F 1..32) form a
 * complete set when veto_a[p][i] == 0, veto_b[p][j] == 0 and neither RSS is NaN; with
 * no track fit to rank them, complete sets are ranked by the combined RSS
 * rss_a[p][i] + rss_b[p][j] (the two sides' wires are disjoint), ascending, ties by
 * the pair index i F + j.
 *   pair       device int32[n_partitions][F F]: i F + j of rank k (-1 past the last)
 *   pair_rss   device double[n_partitions][F F]: its combined RSS (NaN past the last)
 *   n_complete device int32[n_partitions] or NULL: the number of complete sets
 * One block per partition; no allocation. */
int comet_layer_veto(const uint8_t *hit_mask, int64_t mask_stride, int32_t n_rows,
                     const int32_t *row_event, const int32_t *event_wires, int32_t n_events,
                     const int32_t *wire_offsets, const int32_t *wire_layer, int32_t n_wires,
                     int32_t n_layers, int32_t *veto, void *stream);
int comet_merge_halves(const double *rss_a, const int32_t *veto_a, const double *rss_b,
                       const int32_t *veto_b, int32_t n_partitions, int32_t n_seeds,
                       int32_t *pair, double *pair_rss, int32_t *n_complete, void *stream);

/* ------------------------------------------------------------ stage loop (Sec. 3.1)
 * Turn partitions are reconstructed one stage at a time from the last turn backwards.
 * After a stage the hits it classified are left out of later scans, the chosen seed
 * is extrapolated backwards to the previous turn's entry, which gives the next
 * stage's longitudinal seed (z, p_z) (the transverse seed comes from elsewhere: the
 * Hough transform in the paper), and an event stops when fewer than a minimum of
 * wires remain or enough tracks were found. All arrays are device arrays; every call
 * launches on `stream` without allocating or synchronising.
 *
 * comet_backward_seeds: for seed i (seeds6[i][6], at a turn's outward crossing of
 * r = radius mm) the track runs backwards (momentum and charge flipped, the RK4 step
 * of comet_extrapolate_seeds with cfg's field and step) for at most max_steps steps;
 * out6[i] is the state at the first inward crossing of r = radius after an outward
 * one (the previous turn's entry), interpolated linearly in r^2 - radius^2 between
 * the two states of the crossing step, momentum flipped back; NaN (steps[i] = -1)
 * when there is none within max_steps. steps (int32[n]) may be NULL.
 *
 * comet_stage_grids: grids[i][14] = the descriptor of comet_seed_grid with reference
 * state (x, y, z, px, py, pz) = (transverse6[i][0], [1], ext6[i][2], transverse6[i][3],
 * [4], ext6[i][5]), centres (0, |p|, 0, 0) and half-spans half (host double[4]).
 *
 * comet_exclude_hits: the packed events (CSR as in comet_batch_scan, with hit_ids[j] the
 * caller's index of hit j) without the hits whose exclude[j] != 0, and without the
 * wires left with no hit; the order of what remains is kept. Outputs have the input
 * capacities (n_wires + 1, n_hits, n_wires x 6, n_hits); workspace >=
 * comet_exclude_workspace_bytes(n_events), 256-byte aligned. Outputs must not alias
 * inputs.
 *
 * comet_stage_record: for each event e with active[e] != 0, the hits with bit 0 set
 * in hit_mask[e] (indexed as in comet_batch_scan) get stage_of_hit[hit_ids[j]] = stage
 * and exclude[j] = 1; every other hit gets exclude[j] = 0.
 *
 * comet_stage_update: active[e] stays 1 only if best[e] >= 0, stage + 1 <
 * min(n_turns[e], max_stages) and event e keeps at least min_wires wires in the CSR
 * event_wires_next (after the exclusion).
 *
 * comet_self_refine: the self-refining of a stage's classified hits (Sec. 3.1). The
 * paper re-fits the best complete set with a Kalman-type filter, drops hits the fit
 * weights down, and re-examines the hits of wires left without a classified hit
 * against the fitted track with a second cutoff eta (0.3 mm in the paper). Here the
 * fitted track is the track of seeds6[r] (row r's fitted seed, e.g. the chosen seed
 * after comet_lm_refine; host-side layout double[n_rows][6], device memory), extrapolated
 * as comet_extrapolate_seeds does with cfg's field, step and n_steps (<= 2400). For
 * every wire of event row_event[r] (CSR as in comet_batch_scan), with D its DCA to
 * that track:
 *   - a hit with bit 0 set in mask_in[r] stays classified iff |D - r_j| < lambda;
 *   - on a wire where none stays, the hit with the smallest |D - r_j| (first on
 *     ties) is classified iff that residual is below eta.
 * mask_out[r][j - first hit of the event] = 1 for a classified hit, else 0; masks are
 * uint8 [n_rows][mask_stride] and hits past mask_stride are left alone; mask_out may
 * equal mask_in. A seed with a NaN component keeps bit 0 of mask_in. A row whose
 * row_event is outside [0, n_events) is skipped. eta must be finite and >= 0
 * (0: no re-admission). One block per row; no allocation. */
int comet_backward_seeds(const double *seeds6, int32_t n, const comet_config *cfg, double radius,
                         int32_t max_steps, double *out6, int32_t *steps, void *stream);
int comet_stage_grids(const double *transverse6, const double *ext6, int32_t n,
                      const double half[4], double *grids, void *stream);
/* The seed's z as a fifth grid axis (Sec. 3.1: the seed has five degrees of freedom):
 * grids[i][u][14] for u < n_z is comet_stage_grids' descriptor of seed i with the
 * reference z replaced by ext6[i][2] + z_half (2u - (n_z - 1)) / (n_z - 1) (the axis
 * rule of comet_seed_grid; ext6[i][2] itself when n_z = 1). n, n_z >= 1; z_half finite
 * and >= 0; grids device double[n][n_z][14]. */
int comet_stage_grids_z(const double *transverse6, const double *ext6, int32_t n,
                        const double half[4], int32_t n_z, double z_half, double *grids,
                        void *stream);
size_t comet_exclude_workspace_bytes(int32_t n_events);
int comet_exclude_hits(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                       int32_t n_wires, const double *drift, const double *wire_ends,
                       const int32_t *hit_ids, int32_t n_hits, const uint8_t *exclude,
                       int32_t *event_wires_out, int32_t *wire_offsets_out, double *drift_out,
                       double *wire_ends_out, int32_t *hit_ids_out, void *workspace,
                       size_t workspace_bytes, void *stream);
int comet_stage_record(const uint8_t *hit_mask, int64_t mask_stride, int32_t n_events,
                       const int32_t *event_wires, const int32_t *wire_offsets,
                       const int32_t *hit_ids, const int32_t *active, int32_t stage,
                       int32_t *stage_of_hit, uint8_t *exclude, void *stream);
int comet_self_refine(const double *seeds6, int32_t n_rows, const int32_t *row_event,
                      const comet_config *cfg, const double *wire_ends, int32_t n_wires,
                      const int32_t *wire_offsets, const double *drift, int32_t n_hits,
                      const int32_t *event_wires, int32_t n_events, double eta,
                      const uint8_t *mask_in, uint8_t *mask_out, int64_t mask_stride,
                      void *stream);
int comet_stage_update(int32_t *active, int32_t n_events, const int64_t *best,
                       const int32_t *event_wires_next, const int32_t *n_turns, int32_t stage,
                       int32_t max_stages, int32_t min_wires, void *stream);

/* ------------------------------------------------------------ per-stage chain
 * The paper's stage (Sec. 3.1) scans the turn partition as two half tracks, each with
 * several references, vetoes and merges the half sets, self-refines the best complete
 * set and extrapolates backwards from it. The scans, selections, veto, merge,
 * self-refining and backward extrapolation are the entry points above; these four join
 * them. All launch on `stream` without allocating or synchronising.
 *
 * comet_exit_seeds: the exit half track's seed. For state i (states + i row_stride, six
 * doubles (x, y, z, px, py, pz) at a turn's outward crossing of r = radius mm; a
 * row_stride of 14 reads the reference state of comet_seed_grid descriptors) the track
 * runs forwards (the RK4 step of comet_extrapolate_seeds with cfg's field, charge and
 * step) for at most max_steps steps; out6[i] is the state where it first crosses
 * r = radius inwards after having been outside (the turn's re-entry into the seed
 * region), interpolated linearly in r^2 - radius^2 between the crossing step's two
 * states, with the momentum reversed: the exit half is scanned backwards through the
 * turn, with the charge reversed too. NaN (steps[i] = -1) without such a crossing.
 * steps (int32[n]) may be NULL.
 *
 * comet_half_split: per hit j of the packed events (CSR as in comet_batch_scan with
 * hit_ids, as comet_exclude_hits writes them; only the first
 * wire_offsets[event_wires[n_events]] of the n_hits capacity are read) the side of its
 * wire: entrance_side[hit_ids[j]] (uint8[n_ids], nonzero = the entrance half: the
 * turn's hits on the entrance side of the line through the chamber axis and the
 * circle's centre) gives exclude_entrance[j] = 0 and exclude_exit[j] = 1, and the
 * opposite for the exit side; an id outside [0, n_ids) leaves both halves. With
 * comet_exclude_hits the two masks give the halves' CSRs.
 *
 * comet_wire_layers: wire_layer[w] = hit_layer[hit_ids[first hit of wire w]] for the
 * wires of packed events whose every wire holds a hit (comet_exclude_hits output), -1
 * for an id outside [0, n_ids); for comet_layer_veto.
 *
 * comet_union_halves: per event e with active[e] != 0, the best complete set: entrance
 * seed i and exit seed j from pair[e][0] = i n_final + j of comet_merge_halves when
 * n_complete[e] > 0, else (0, 0), the lowest-RSS final seed of each side. Its hits:
 * mask_out[e][k] (k the hit's index within event e of the packed events, which hold
 * both halves' hits) is bit 0 of mask_a[e n_final + i] at the hit's index among the
 * event's entrance hits, or of mask_b[e n_final + j] among its exit hits; seed_out[e] =
 * seeds_a[e n_final + i] (double[6]); best_out[e] = i n_final + j, or -1 when that
 * seed is NaN. Inactive events get seed_out NaN and best_out -1 and keep mask_out.
 * n_final in 1..64; masks uint8 [rows][stride]. One wave per event. */
int comet_exit_seeds(const double *states, int64_t row_stride, int32_t n, const comet_config *cfg,
                     double radius, int32_t max_steps, double *out6, int32_t *steps,
                     void *stream);
int comet_half_split(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                     const int32_t *hit_ids, int32_t n_hits, const uint8_t *entrance_side,
                     int32_t n_ids, uint8_t *exclude_entrance, uint8_t *exclude_exit,
                     void *stream);
int comet_wire_layers(const int32_t *event_wires, int32_t n_events, const int32_t *wire_offsets,
                      int32_t n_wires, const int32_t *hit_ids, const int32_t *hit_layer,
                      int32_t n_ids, int32_t *wire_layer, void *stream);
int comet_union_halves(const int32_t *pair, const int32_t *n_complete, int32_t n_final,
                       int32_t n_events, const int32_t *event_wires, const int32_t *wire_offsets,
                       const int32_t *hit_ids, const uint8_t *entrance_side, int32_t n_ids,
                       const uint8_t *mask_a, int64_t stride_a, const uint8_t *mask_b,
                       int64_t stride_b, const double *seeds_a, const int32_t *active,
                       uint8_t *mask_out, int64_t stride_out, double *seed_out,
                       int64_t *best_out, void *stream);

/* Shapes of the batched scan kernel (W wires per wave, NWV waves per block, C points
 * per LDS chunk, the persistent block count on the current device, and direct and runs
 * as for the DCA shapes, with direct = 4 for the wide form with the residual cap whose
 * waves take each event's wires in azimuth order (events of more than 3 (n_steps + 1)
 * wires in wire order) and 5 for that form with the first index of each minimum
 * tracked point by point (five shapes also testing each half or quarter of a needed
 * chunk per wire, every test from the middle of its stretch, two of them taking each
 * tile as a 2 x 2 x 4 x 4 block of the grid);
 * blocks, direct and runs may be NULL); every shape gives the same results.
 * comet_batch_set_variant selects the shape (default 0). */
int comet_batch_variant_count(void);
int comet_batch_variant_info(int id, int32_t *w, int32_t *nwv, int32_t *chunk, int32_t *blocks,
                             int32_t *direct, int32_t *runs);
int comet_batch_set_variant(int id);

/* ------------------------------------------------------------ diagnostics
 * Per-kernel device time. After comet_profile_begin() every kernel launched by the
 * calls above is bracketed by two HIP events recorded on its stream (the events are
 * created on first use and reused afterwards; recording adds no synchronisation).
 * comet_profile_end() waits for the recorded events, writes per kernel kind the
 * summed duration in milliseconds and the number of launches, and stops recording.
 * Kinds: 0 track recording, 1 DCA scan, 2 RSS sum, 3 selection and classification.
 * Both return COMET_OK or COMET_EHIP; profiling state is process-wide. */
#define COMET_PROFILE_KINDS 4
int comet_profile_begin(void);
int comet_profile_end(double ms[COMET_PROFILE_KINDS], int64_t launches[COMET_PROFILE_KINDS]);
/* The number of (seed, wire, track point) distance evaluations the DCA scans (single
 * event and batched) performed on the device current at comet_profile_begin, between
 * it and the last comet_profile_end (the scans skip points a distance bound rules
 * out, so this is at most seeds x wires x points per scan). COMET_EINVAL for NULL. */
int comet_profile_scan_points(int64_t *points);

/* ------------------------------------------------------------ tuning
 * The DCA kernel exists in several shapes: W wires per wave, NWV waves per block,
 * C track points per LDS chunk, whether the first closest index is tracked per point
 * (chunk_argmin = 0) or per chunk with a final rescan (1), whether blocks are
 * remapped so that one seed tile's wire groups share an XCD, and whether the block's
 * waves share the needed chunks through LDS (direct = 0) or each wave loads the
 * chunks it needs itself, with no LDS and no barrier (direct = 1). Every shape gives
 * the same results bit for bit; only speed differs.
 *
 * comet_dca_autotune() takes the arguments of comet_dca_rss (same checks, same
 * result in rss) plus: reps (1..1000) timed launches per shape, best_id (host, may be
 * NULL) receiving the chosen shape, ms (host, may be NULL, comet_dca_variant_count()
 * entries) receiving each shape's mean kernel time. It chooses, among the shapes
 * within 1 % of the fastest, the one with the fewest wire groups (each group reads
 * the seed tile's track once more), records it for this (n_seeds, n_points, n_wires),
 * and later comet_dca_rss calls of that size use it. Unlike the other calls it creates two HIP events and synchronises `stream`: it
 * is a set-up call, not one for a timed loop.
 *
 * comet_dca_set_variant(id) forces shape id for every call (-1 removes the override);
 * comet_dca_variant_for() reports the shape a call of that size would use;
 * comet_dca_variant_info() describes shape id (0 <= id < comet_dca_variant_count()):
 * W wires per wave, NWV waves per block, chunk points, per-chunk argmin, XCD-aware
 * block order, direct (0: the block's chunks staged through LDS; 1: every wave on its
 * own, no LDS staging; 2: wide, every wave on its own with up to 16 wires taken in
 * azimuth order, frames in LDS, each wire of a needed chunk scanned only where the
 * bound needs it; 3: wide with Eq. 1's residual cap in the bound; 5: that form with the
 * first index of each minimum tracked point by point, so that the end reads only the
 * chord refinement's points, some shapes also testing each half or quarter of a needed
 * chunk per wire before scanning it) and runs (direct and
 * wide shapes: chunks tested in runs of that many first, from the summed radii of their
 * windows; 1 = no runs); direct and runs may be NULL. comet_dca_variant_name(id): the
 * shape's kernel as a profiler names it ("" for an id out of range). */
int comet_dca_variant_count(void);
int comet_dca_variant_info(int id, int32_t *w, int32_t *nwv, int32_t *chunk,
                           int32_t *chunk_argmin, int32_t *xcd_remap, int32_t *direct,
                           int32_t *runs);
const char *comet_dca_variant_name(int id);
int comet_dca_set_variant(int id);
int comet_dca_variant_for(int64_t n_seeds, int32_t n_points, int32_t n_wires);
int comet_dca_autotune(const double *track_xyz, int64_t n_seeds, int32_t n_points,
                       const double *wire_ends, int32_t n_wires, const int32_t *wire_offsets,
                       const double *drift, int32_t n_hits, const comet_config *cfg, double *rss,
                       void *workspace, size_t workspace_bytes, int32_t reps, int32_t *best_id,
                       double *ms, void *stream);

/* Static description of a status code. */
const char *comet_status_string(int status);

/* Details of the last failure on the calling thread ("" if none). */
const char *comet_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int comet_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COMET_H */
