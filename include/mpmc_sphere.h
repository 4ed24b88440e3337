/*
 * mpmc_sphere.h -- C ABI of libmpmc.so for hard SPHERES in three dimensions:
 * the same massively parallel Metropolis chain as mpmc.h, for d = 3.
 *
 * Method: Anderson, Jankowski, Grubb, Engel, Glotzer, arXiv:1211.1646.  The
 * paper states its scheme for d dimensions (Sec. 2): cells of width
 * w >= sigma, 2^d checkerboard sets processed in a random order (Alg. 1),
 * every active cell updating only its own particles with trial moves that
 * must stay inside the cell and overlap nothing in the 3^d neighbourhood
 * (Alg. 2), and a random shift of the cell grid along one axis at the end
 * of a sweep (Sec. 3.2, Alg. 4).  In three dimensions:
 *  - cubic cells with 1 <= w < 2/sqrt(3) per axis, so at most 8 centres fit
 *    in a cell (the cube's corners; a ninth needs w >= 2/sqrt(3)): the
 *    capacity is 8;
 *  - 8 checkerboard sets, set Q = (cx & 1) + 2 (cy & 1) + 4 (cz & 1), cells
 *    numbered c = (cz m_y + cy) m_x + cx;
 *  - the 27-cell neighbourhood, with pair distance
 *    r^2 = fmaf(dz, dz, fmaf(dy, dy, dx*dx)) in FP32 (one rounding per
 *    added square), overlap iff r^2 < 1;
 *  - 6 shift directions f = +x, -x, +y, -y, +z, -z (0..5).
 *
 * Random numbers (Philox4x32-10, key (seed, replica), counter (cell or
 * 0xFFFFFFFF, sweep low word, sweep high word, tag)):
 *  - trial t of a cell update uses words 2(t&1) and 2(t&1)+1 of the cell's
 *    block with tag t >> 1: x from the high and y from the low half of the
 *    first word, z from the high half of the second; a half h gives the
 *    displacement (2h + 1 - 65536) / 65536 * delta;
 *  - the particle shuffle (Fisher-Yates over the stored list, i = n-1..1,
 *    j = floor(u (i+1) / 2^32)) takes word k & 3 of the block with tag
 *    0x40000000 + (k >> 2) for its k-th step;
 *  - sweep s orders the 8 sets by Fisher-Yates (i = 7..1) with words
 *    u0..u6 of the global blocks with tags 0x80000000 (u0..u3) and
 *    0x80000001 (u4..u7), picks f = floor(u7 6 / 2^32) and
 *    d = (low 24 bits of word 0 of the block with tag 0x80000002) 2^-24 w_f/2.
 *
 * Conventions are those of mpmc.h: the caller owns the device buffers (sizes
 * from mpmc_sphere_required_bytes, each 256-byte aligned), `stream` is a
 * hipStream_t passed as void*, calls are "async" (enqueue only) or "sync"
 * (wait and copy to host), every call returns MPMC_OK or a negative
 * MPMC_E* status with a message from mpmc_last_error(), and a kernel that
 * finds a cell above capacity sets an error word that the next sync call
 * reports as MPMC_EDEVICE.  Positions are FP32 cell-local coordinates in
 * (0, w] per axis; the state calls exchange them as compact lists (cells in
 * the order above, the spheres of cell c at xyz[3k .. 3k+2] for
 * start[c] <= k < start[c+1], start[cells] = N).  One handle holds one system.
 */
#ifndef MPMC_SPHERE_H
#define MPMC_SPHERE_H

#include "mpmc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MPMC_SPHERE_CAPACITY 8

typedef struct mpmc_sphere *mpmc_sphere_handle;

/* System description; sigma = 1. */
typedef struct mpmc_sphere_params {
    int32_t lattice_nx;  /* > 0: start from an nx x ny x nz simple cubic lattice */
    int32_t lattice_ny;  /*      at packing fraction eta = N pi / (6 V)          */
    int32_t lattice_nz;
    double eta;          /*      0 < eta <= pi/6                                  */
    int32_t cells_x;     /* > 0: explicit even cell counts (>= 4); 0: smallest    */
    int32_t cells_y;     /*      even count with w < w_max                         */
    int32_t cells_z;
    double w_max;        /* 0 or >= 2/sqrt(3): the capacity limit 2/sqrt(3)       */
    float cell_w_x;      /* lattice_nx == 0: explicit cell widths; the state is   */
    float cell_w_y;      /*   then loaded with mpmc_sphere_set_state              */
    float cell_w_z;
    int64_t n_particles; /* lattice_nx == 0: particle count to size buffers      */
    float delta;         /* trial displacement uniform in (-delta, delta)^3;      */
                         /*   0 < delta <= min(w)/2                               */
    int32_t n_moves;     /* n_M: trial moves per active cell per sub-sweep, >= 0  */
    uint32_t seed;       /* Philox key word 0                                     */
    uint32_t replica;    /* Philox key word 1                                     */
    uint32_t flags;      /* MPMC_FLAG_TAG (identity tags), MPMC_FLAG_ACC          */
                         /*   (displacement accumulators), or 0                   */
} mpmc_sphere_params;

/* Derived geometry.  The lattice's site (i, j, k) sits at
 * ((i + 1/4) a, (j + 1/4) a, (k + 1/4) a), a = (pi / (6 eta))^(1/3), in
 * cell ceil(x / w) - 1 per axis; cells list their spheres in ascending
 * lattice index (k n_y + j) n_x + i. */
typedef struct mpmc_sphere_geometry {
    int64_t n_particles;
    int32_t cells_x, cells_y, cells_z;
    float w_x, w_y, w_z;       /* FP32 cell widths: the dynamics' box is cells * w */
    double box_x, box_y, box_z;
    double density;            /* n_particles / (box_x box_y box_z)               */
} mpmc_sphere_geometry;

/* Device buffer sizes.  pos, count and tag are ping-pong pairs: each half
 * needs the reported size.  On the device the spheres sit in fixed slots,
 * MPMC_SPHERE_CAPACITY per cell, as float4 (x, y, z, 0), with a uint32
 * count per cell: slots 0..1 of cell c in its 32-byte primary line, slots
 * 2..7 in an overflow region after all primary lines.  The fourth word of
 * slot 0 repeats the cell's count (its bits), so that the sub-sweep reads a
 * cell's count and first two spheres from one line. */
typedef struct mpmc_sphere_buffer_sizes {
    size_t pos;   /* float4 per slot (cells x 8)                 */
    size_t count; /* uint32 per cell                             */
    size_t tag;   /* uint32 per slot (MPMC_FLAG_TAG), else 0     */
    size_t acc;   /* float4 per slot (MPMC_FLAG_ACC), else 0     */
    size_t work;  /* counter partials, MSD partials              */
    size_t ctl;   /* control block: sweep counter, key, delta,
                     counters, error word, contact histogram     */
} mpmc_sphere_buffer_sizes;

typedef struct mpmc_sphere_buffers {
    void *pos[2];
    void *count[2];
    void *tag[2];  /* NULL unless MPMC_FLAG_TAG */
    void *acc[2];  /* NULL unless MPMC_FLAG_ACC */
    void *work;
    void *ctl;
} mpmc_sphere_buffers;

/* Geometry of a parameter set (Sec. 3.1 in d = 3; host only).  Errors: MPMC_EINVAL for a bad
 * lattice, eta, delta, n_moves or flags; MPMC_EGEOM for cell counts that are
 * odd or below 4, or widths outside [1, 2/sqrt(3)). */
mpmc_status mpmc_sphere_geometry_of(const mpmc_sphere_params *p, mpmc_sphere_geometry *out);

/* Utility: buffer sizes for a parameter set (host only). */
mpmc_status mpmc_sphere_required_bytes(const mpmc_sphere_params *p,
                                       mpmc_sphere_buffer_sizes *out);

/* Build the system (N spheres at packing fraction eta; the method in
 * d = 3, Sec. 2.1) and upload it on `stream` (sync): the lattice when
 * lattice_nx > 0, else an empty grid to be filled by mpmc_sphere_set_state.
 * Sweep 0, counters 0, delta and key from p. */
mpmc_status mpmc_sphere_init(const mpmc_sphere_params *p, const mpmc_sphere_buffers *b,
                             void *stream, mpmc_sphere_handle *out);

/* n_sweeps sweeps (async): the sweep's set order, eight sub-sweeps, shift
 * and rebin, sweep += 1 (Alg. 1 in d = 3).  Long runs are launched as
 * captured hipGraphs of a fixed block of sweeps. */
mpmc_status mpmc_sphere_sweep(mpmc_sphere_handle h, int64_t n_sweeps);

/* One sub-sweep of set `set` (0..7) with the current sweep's cell streams
 * (Alg. 2 in d = 3).  async. */
mpmc_status mpmc_sphere_subsweep(mpmc_sphere_handle h, int32_t set);

/* Shift and rebin (Alg. 4 in d = 3).  f in 0..5 with 0 <= d <= w_f / 2
 * shifts by that amount and keeps the sweep counter; f = -1 takes f and d
 * from the current sweep's draws and advances the sweep counter.  New cell c
 * lists the spheres of old c that stay, then those of its neighbour in
 * direction f that move in, both in stored order.  async. */
mpmc_status mpmc_sphere_shift(mpmc_sphere_handle h, int32_t f, float d);

/* Utility (state transfer): copy the state to host memory (sync): xyz[3N], start[cells + 1], tags[N]
 * (MPMC_FLAG_TAG), sweep counter.  Any pointer may be NULL. */
mpmc_status mpmc_sphere_get_state(mpmc_sphere_handle h, float *xyz, uint32_t *start,
                                  uint32_t *tags, uint64_t *sweep);

/* Utility (state transfer): load a state (sync).  Offsets, capacity and coordinate ranges are checked
 * on the host (MPMC_ESTATE), overlaps on the device (MPMC_EOVERLAP); tags may
 * be NULL (then 0..N-1 in list order).  Counters restart at 0. */
mpmc_status mpmc_sphere_set_state(mpmc_sphere_handle h, const float *xyz, const uint32_t *start,
                                  uint64_t sweep, const uint32_t *tags);

/* Trial moves (counted by the paper's throughput eta, Sec. 5) and accepted
 * moves since init or set_state (sync). */
mpmc_status mpmc_sphere_get_counters(mpmc_sphere_handle h, uint64_t *trials, uint64_t *accepts);

/* Maximum trial displacement, the free parameter d of Sec. 3.3 (async set, 0 < delta <= min(w)/2; sync get). */
mpmc_status mpmc_sphere_set_delta(mpmc_sphere_handle h, float delta);
mpmc_status mpmc_sphere_get_delta(mpmc_sphere_handle h, float *delta);

/* Plain acceptance tuner for equilibration (async): n_windows times, run
 * window_sweeps sweeps, then with a = accepts/trials of that window set
 * delta <- delta * clamp(a/0.3, 0.5, 2) in FP64, clamped to
 * [1e-3, min(w)/2] and rounded once to FP32, on the device.  delta is a free
 * parameter of the method (Sec. 3.3); freeze it (stop tuning) before
 * sampling.  window_sweeps >= 1, n_windows >= 0. */
mpmc_status mpmc_sphere_tune(mpmc_sphere_handle h, int32_t window_sweeps, int32_t n_windows);

/* Accumulate the ordered-pair contact histogram of the current
 * configuration (Sec. 4's estimator in d = 3: 200 bins of width 1e-4 on
 * [1, 1.02), binned on FP32 r^2 edges (float)((1 + b 1e-4)^2)).  reset != 0
 * clears it first.  async.  MPMC_EGEOM if a cell count is too small for
 * the histogram's reach (six cells per axis when w < 1.02). */
mpmc_status mpmc_sphere_pair_histogram(mpmc_sphere_handle h, int32_t reset);

/* Pressure from the contact value (sync): g(R_i) = n_i / (S N rho 4 pi R_i^2
 * dr) at the volume-weighted shell radii R_i = 3/4 (r1^4 - r0^4) /
 * (r1^3 - r0^3), g(sigma+) from an unweighted degree-5 least-squares fit in
 * (R - 1)/0.02, and beta P sigma^3 = rho (1 + 2 pi/3 rho g(sigma+)), all in
 * FP64 on the device from the accumulated histogram (the current
 * configuration's if none).  Any output may be NULL; hist receives
 * MPMC_HIST_BINS counts. */
mpmc_status mpmc_sphere_pressure(mpmc_sphere_handle h, double *p_star, double *g_contact,
                                 uint64_t *hist, uint64_t *n_samples);

/* Utility (invariant check: hard spheres never overlap): ordered pairs
 * closer than 1 - 2^-20 in squared distance (sync). */
mpmc_status mpmc_sphere_count_overlaps(mpmc_sphere_handle h, int64_t *pairs);

/* Utility (performance only): launch shape of the sub-sweep: 1, 2 or 4
 * lanes per active cell (default 1).  With one lane per cell a workgroup
 * stages a brick of 4 x 4 x 4 active cells and their neighbours in LDS (the
 * per-lane form when accumulators are on); with 2 or 4 the lanes of a group
 * split the 26 neighbour cells and their overlap tests and combine their
 * verdicts.  Every comparison is the same, so the results do not depend on
 * it (sync: waits for the stream, drops the sweep graphs). */
mpmc_status mpmc_sphere_set_launch(mpmc_sphere_handle h, int32_t lanes_per_cell);

/* Utility, not in the paper (diffusion measure): displacement accumulators
 * (MPMC_FLAG_ACC): every accepted move adds its
 * displacement, one FP32 add per axis, to its sphere's accumulator, which
 * follows the sphere through shuffles and shifts; init, set_state and
 * reset_acc zero them.  get_acc copies acc[3N] in list order (sync); msd
 * gives mean |acc|^2 over the spheres, FP64 in a fixed order (sync);
 * reset_acc zeroes them (async).  MPMC_EINVAL without the flag. */
mpmc_status mpmc_sphere_get_acc(mpmc_sphere_handle h, float *acc);
mpmc_status mpmc_sphere_msd(mpmc_sphere_handle h, double *msd);
mpmc_status mpmc_sphere_reset_acc(mpmc_sphere_handle h);

/* Utility: wait for the handle's work; reports MPMC_EDEVICE for a set error
 * word. */
mpmc_status mpmc_sphere_synchronize(mpmc_sphere_handle h);

/* Utility: free the handle and its graphs (not the caller's buffers). */
void mpmc_sphere_destroy(mpmc_sphere_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MPMC_SPHERE_H */
