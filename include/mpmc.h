/*
 * mpmc.h -- C ABI of libmpmc.so: massively parallel Metropolis Monte Carlo of
 * hard disks on one AMD Instinct MI355X (gfx950).
 *
 * Method: Anderson, Jankowski, Grubb, Engel, Glotzer, "Massively parallel
 * Monte Carlo for many-particle simulations on GPUs" (arXiv:1211.1646).
 * A sweep (Alg. 1) shuffles the four checkerboard sets of cells (Eq. 1),
 * updates every cell of one set concurrently -- shuffle the cell's particles,
 * then n_M trial moves on particle list[s mod n], rejecting moves that leave
 * the cell or overlap a disk of the 3x3 neighbourhood (Alg. 2; in FP32,
 * r^2 = fmaf(dy, dy, dx*dx) < 1) -- and ends with a random shift of the cell
 * grid (Alg. 4).
 *
 * Conventions for every call:
 *  - Device memory is owned by the caller.  mpmc_required_bytes() reports the
 *    size of each buffer; the caller allocates them (e.g. as torch tensors)
 *    and passes device pointers in mpmc_buffers.  The library keeps non-owning
 *    pointers that must stay valid until mpmc_destroy().  The library itself
 *    allocates only its small host-side handle and, for mpmc_sweep, the
 *    hipGraph objects it captures.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls marked "async" only enqueue work on it; calls marked "sync" wait
 *    for it and copy results to host memory.
 *  - Positions are FP32 cell-local coordinates in (0, w] per axis.  The
 *    state calls exchange them in compressed-row form: cells in row-major
 *    order c = cy*cells_x + cx, the particles of cell c at xy[2*k],
 *    xy[2*k+1] for start[c] <= k < start[c+1], start[cells] = N.  (The
 *    device buffers hold them in per-cell slots; see mpmc_buffer_sizes.)
 *  - Every call returns MPMC_OK (0) or a negative status; mpmc_last_error()
 *    gives a message for the calling thread's last failure.  Argument and
 *    geometry errors are detected on the host before anything is enqueued.
 *    Invariant violations found by a kernel (a cell above capacity) set a
 *    device error word that the next sync call reports as MPMC_EDEVICE.
 *  - The random streams are Philox4x32-10 with key (seed, replica) and
 *    counter (cell or 0xFFFFFFFF, sweep low word, sweep high word, tag); the
 *    sweep counter lives in device memory, so results depend only on the
 *    state, the sweep index and the key -- not on launch shapes.
 *  - A handle holds R >= 1 independent systems ("replicas"), each with its
 *    own N, packing fraction, grid, delta, n_M, key and sweep counter.
 *    mpmc_init_system builds R = 1; mpmc_batch_init builds R >= 1.  Calls
 *    that advance the chain (sweep, subsweep, shift_and_rebin, tune,
 *    pair_histogram, reset_acc, set_delta) act on every replica at once,
 *    in the same kernel launches; replica r then evolves exactly as a single
 *    system with the same parameters would.  The per-system getters without
 *    a replica argument require R = 1 (MPMC_EINVAL otherwise); the
 *    mpmc_replica_* forms take the replica index.
 */
#ifndef MPMC_H
#define MPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mpmc_status;
#define MPMC_OK 0
#define MPMC_EINVAL (-1)   /* bad argument */
#define MPMC_EGEOM (-2)    /* grid odd or < 4 cells, w < sigma, w too wide for capacity 7 */
#define MPMC_EOVERLAP (-3) /* state handed in contains overlapping disks */
#define MPMC_EHIP (-4)     /* HIP runtime error */
#define MPMC_EDEVICE (-5)  /* a kernel found an invariant violation */
#define MPMC_ESTATE (-6)   /* state handed in is malformed (offsets, ranges, capacity) */

#define MPMC_FLAG_ACC 1u   /* keep per-disk displacement accumulators (MSD) */
#define MPMC_FLAG_TAG 2u   /* keep per-disk identity tags */
#define MPMC_FLAG_ACCEPT_LOG 4u /* keep per-cell accept bits of the latest update */
/* Trial displacements uniform in the disk of radius delta, the paper's
 * inCircle(d) proposal (Alg. 2), instead of the square (-delta, delta)^2.
 * One trial word still makes one move: its high half gives the squared
 * radius (2h+1)/2^17 of the disk, its low half the angle (2h+1) pi/65536,
 * evaluated with FP32 Taylor series about 0 on (0, pi/4) and exact quarter
 * turns.  The proposal is exactly symmetric.  Replicas of one batch may
 * differ in this flag and in the two below; the buffer flags above must
 * agree. */
#define MPMC_FLAG_DISK 8u
/* Diagnostics, for the balance test of Sec. 2.4 (Table 1): switch off the
 * shuffle of each cell's particle list (cells are then visited in stored
 * order, which breaks detailed balance), or the shuffle of the order of the
 * four checkerboard sets (always a, b, c, d; the paper finds this harmless).
 * All other random draws are unchanged.  Replicas may differ in them. */
#define MPMC_FLAG_NO_PARTICLE_SHUFFLE 16u
#define MPMC_FLAG_NO_SET_SHUFFLE 32u
/* Diagnostics, the two cell-leaving pitfalls of Sec. 2.4 (they break
 * detailed balance): LEAVE lets a move take its disk out of the cell, by
 * at most e = (w - 1)/2 per axis (so that the 3x3 overlap test stays
 * complete and the cells of one set independent); the disk stays in its
 * cell's list until the sweep's shift re-homes it on both axes.
 * LEAVE_ONCE is LEAVE with n_M = n for every cell update, each disk moved
 * exactly once per sweep.  The shift then lists, in new cell c, its own
 * stayers and then the arrivals from the eight neighbours in row-major
 * order of the offset.  Replicas may differ in them.  Sweeps of a handle
 * with either flag use the separate launches, one lane per cell. */
#define MPMC_FLAG_LEAVE 64u
#define MPMC_FLAG_LEAVE_ONCE 128u

#define MPMC_HIST_BINS 200 /* contact histogram: 200 bins of 1e-4 sigma */

typedef struct mpmc_system *mpmc_handle;

/* System description (Sec. 3.1 and 3.3 free parameters: cell width via the
 * grid, maximum move delta, moves per cell n_M, seed).  sigma = 1. */
typedef struct mpmc_params {
    int32_t lattice_nx;  /* > 0: start from an nx x ny triangular lattice      */
    int32_t lattice_ny;  /*      (ny even) at packing fraction phi            */
    double phi;
    int32_t cells_x;     /* > 0: explicit grid; 0: chosen from w_min / w_max  */
    int32_t cells_y;
    double w_min;        /* largest even grid with width >= w_min (default 1) */
    double w_max;        /* > 0: smallest even grid with width < w_max         */
    float cell_w_x;      /* lattice_nx == 0: explicit cell widths; the state  */
    float cell_w_y;      /*   is then loaded with mpmc_set_state              */
    int64_t n_particles; /* lattice_nx == 0: particle count to size buffers   */
    float delta;         /* trial displacement uniform in (-delta, delta)^2;  */
                         /*   0 < delta <= min(w)/2                           */
    int32_t n_moves;     /* n_M: trial moves per active cell per sub-sweep    */
    uint32_t seed;       /* Philox key word 0                                 */
    uint32_t replica;    /* Philox key word 1                                 */
    uint32_t flags;      /* MPMC_FLAG_*                                       */
} mpmc_params;

/* Derived geometry (Sec. 3.1; capacity from Fig. 3). */
typedef struct mpmc_geometry {
    int64_t n_particles;
    int32_t cells_x, cells_y;
    float w_x, w_y;        /* FP32 cell widths: the dynamics' box is cells*w   */
    int32_t capacity;      /* most disks one cell can hold (4..7)             */
    double box_x, box_y;   /* cells_x * w_x, cells_y * w_y (FP64)              */
    double density;        /* n_particles / (box_x * box_y)                    */
} mpmc_geometry;

/* Bytes the caller must provide for each buffer.  pos/count/acc/tag are
 * ping-pong pairs: each of the two halves needs the reported size.  acc and
 * tag are 0 unless the corresponding flag is set.  On the device the disks
 * sit in fixed slots, capacity-many per cell (the paper's disk[x, y, i],
 * Sec. 3.1; the largest capacity of a batch's replicas), with a count per
 * cell; the state calls below exchange compact lists. */
typedef struct mpmc_buffer_sizes {
    size_t pos;   /* float2 per slot (cells x capacity)                        */
    size_t count; /* uint32 per cell                                           */
    size_t acc;   /* float2 per slot (MPMC_FLAG_ACC)                            */
    size_t tag;   /* uint32 per slot (MPMC_FLAG_TAG)                            */
    size_t work;  /* scratch: completion counters, partials, reductions        */
    size_t ctl;   /* control block: sweep counter, key, delta, counters,
                     error word, contact histogram                             */
    size_t accept_log; /* uint32 per cell (MPMC_FLAG_ACCEPT_LOG), else 0        */
} mpmc_buffer_sizes;

/* Device pointers, each 256-byte aligned, sizes as reported above. */
typedef struct mpmc_buffers {
    void *pos[2];
    void *count[2];
    void *acc[2];   /* NULL unless MPMC_FLAG_ACC */
    void *tag[2];   /* NULL unless MPMC_FLAG_TAG */
    void *work;
    void *ctl;
    void *accept_log; /* NULL unless MPMC_FLAG_ACCEPT_LOG */
} mpmc_buffers;

/* Geometry of a parameter set (Sec. 3.1, Fig. 3).  Host only, no GPU use.
 * Errors: MPMC_EINVAL for bad lattice/phi, MPMC_EGEOM for an unusable grid. */
mpmc_status mpmc_geometry_of(const mpmc_params *p, mpmc_geometry *out);

/* Utility (no passage of the method): buffer sizes for a parameter set.
 * Host only, no GPU use. */
mpmc_status mpmc_required_bytes(const mpmc_params *p, mpmc_buffer_sizes *out);

/* Utility: buffer sizes for n_replicas systems, per_replica[0 .. n_replicas).  All
 * replicas must share `flags`.  In the shared layout each replica's cells
 * are padded to a multiple of 256 (at least one padding cell) and its active
 * cells to a multiple of 768.  Host only.  Errors as mpmc_geometry_of, plus MPMC_EINVAL for
 * n_replicas outside [1, 65535] or differing flags, and MPMC_EGEOM when the
 * total exceeds 32-bit offsets. */
mpmc_status mpmc_batch_required_bytes(const mpmc_params *per_replica, int32_t n_replicas,
                                      mpmc_buffer_sizes *out);

/* init_system: build the system (Sec. 4: N disks at packing fraction phi)
 * and upload it on `stream` (sync).  With lattice_nx > 0 the state is the
 * triangular lattice; otherwise the grid is explicit and empty until
 * mpmc_set_state.  Sets sweep = 0, counters = 0, delta and key from p.
 * *out receives a handle to destroy with mpmc_destroy. */
mpmc_status mpmc_init_system(const mpmc_params *p, const mpmc_buffers *b, void *stream,
                             mpmc_handle *out);

/* Batched form: n_replicas independent systems in one handle (sync).  Replica
 * r is built from per_replica[r] exactly as mpmc_init_system would build it
 * (lattice replicas start from their lattice; grid replicas stay empty until
 * mpmc_replica_set_state) and is keyed (seed, replica) from its own params.
 * Buffers are sized by mpmc_batch_required_bytes. */
mpmc_status mpmc_batch_init(const mpmc_params *per_replica, int32_t n_replicas,
                            const mpmc_buffers *b, void *stream, mpmc_handle *out);

/* Utility: number of replicas of a handle. */
mpmc_status mpmc_num_replicas(mpmc_handle h, int32_t *n);

/* Geometry of replica r (Sec. 3.1, Fig. 3; host only). */
mpmc_status mpmc_replica_geometry(mpmc_handle h, int32_t r, mpmc_geometry *out);

/* sweep(n_sweeps, seed): n_sweeps full sweeps of Alg. 1 (async): the sweep's
 * set order, four sub-sweeps (Alg. 2), shift and rebin (Alg. 4), sweep += 1.
 * `seed` replaces key word 0 for these and later sweeps.  On a non-default
 * stream every sweep is launched from a captured hipGraph: floor(n / 16)
 * launches of a 16-sweep graph, then one graph of the n mod 16 rest; the
 * graphs are captured on first use and kept (one of each per ping-pong
 * half) until the launch shape or n_M changes.  On the default stream the
 * kernels are launched one by one.  In a batch this is the batched sweep:
 * one launch per step covers every replica.  Errors: MPMC_EINVAL for a
 * negative count, MPMC_ESTATE without a loaded state, MPMC_EHIP. */
mpmc_status mpmc_sweep(mpmc_handle h, int64_t n_sweeps, uint32_t seed);
/* (In a batch, `seed` replaces key word 0 of every replica; key word 1 stays
 * each replica's own.) */

/* Utility (timing support, no passage of the method): capture, without
 * running anything, the graphs that a following mpmc_sweep(h, n_sweeps, .)
 * will launch, so that call enqueues graph launches only (async; nothing is
 * enqueued).  Errors as mpmc_sweep. */
mpmc_status mpmc_prepare_sweeps(mpmc_handle h, int64_t n_sweeps);

/* One sub-sweep of checkerboard set `set` (0..3 = a..d of Eq. 1) with the
 * current sweep's cell streams (Alg. 1, Alg. 2).  async. */
mpmc_status mpmc_subsweep(mpmc_handle h, int32_t set);

/* shift_and_rebin (Alg. 4).  f in 0..3 (+x, -x, +y, -y) with 0 <= d <= w_f/2
 * shifts by the given amount and leaves the sweep counter alone; f = -1 takes
 * f and d from the current sweep's draws and then advances the sweep counter
 * (the last step of a sweep).  The cell lists are rebuilt into the other
 * ping-pong half by a per-cell gather into fixed slots: new cell c receives
 * the disks of old c that stay (0 < shifted coordinate <= w), in slot order,
 * followed by the disks that leave the old cell on the shift side, in slot
 * order -- Alg. 4's list order, with no scan because every cell owns
 * `capacity` slots.  async. */
mpmc_status mpmc_shift_and_rebin(mpmc_handle h, int32_t f, float d);

/* Accumulate the ordered-pair contact histogram of the current configuration
 * into the control block (Sec. 4: 200 bins of width 1e-4 on [1, 1.02),
 * binned on r^2 edges).  reset != 0 clears the accumulated histogram first.
 * async.  Errors: MPMC_EGEOM if the grid is too small for the histogram's
 * reach (two cells per axis when w < 1.02). */
mpmc_status mpmc_pair_histogram(mpmc_handle h, int32_t reset);

/* pressure_from_contact: P* = rho (1 + pi/2 rho g(sigma+)) (Eq. P), with
 * g(sigma+) from a degree-5 least-squares fit of g(R_i) (Eqs. gR, R) over
 * (1, 1.02], computed on the device in FP64 from the accumulated histogram;
 * if none has been accumulated, the current configuration's.  sync.
 * Any output pointer may be NULL; hist receives MPMC_HIST_BINS counts. */
mpmc_status mpmc_pressure_from_contact(mpmc_handle h, double *p_star, double *g_contact,
                                       uint64_t *hist, uint64_t *n_samples);
/* The same for replica r of a batch, from its own histogram; with R > 1 a
 * replica without an accumulated histogram gives MPMC_ESTATE. */
mpmc_status mpmc_replica_pressure_from_contact(mpmc_handle h, int32_t r, double *p_star,
                                               double *g_contact, uint64_t *hist,
                                               uint64_t *n_samples);

/* Utility (state transfer for checkpoints and tests): copy the state to
 * host memory (sync): xy[2N] local coordinates,
 * start[cells+1], sweep counter.  Any pointer may be NULL. */
mpmc_status mpmc_get_state(mpmc_handle h, float *xy, uint32_t *start, uint64_t *sweep);
/* Replica r's state in its own numbering: xy[2 N_r], start[C_r + 1] with
 * start[0] = 0, its sweep counter (sync). */
mpmc_status mpmc_replica_get_state(mpmc_handle h, int32_t r, float *xy, uint32_t *start,
                                   uint64_t *sweep);

/* Utility (state transfer): load a state from host memory (sync).
 * Validates offsets, per-cell
 * capacity and coordinate ranges on the host (MPMC_ESTATE) and overlaps on
 * the device (MPMC_EOVERLAP); tags may be NULL (then 0..N-1 in list order);
 * accumulators are cleared.  N must equal the n_particles the buffers were
 * sized for. */
mpmc_status mpmc_set_state(mpmc_handle h, const float *xy, const uint32_t *start,
                           uint64_t sweep, const uint32_t *tags);
/* Load replica r's state (own numbering, N_r disks) and reset its sweep
 * counter, counters, delta and key to its initial ones (sync).  The other
 * replicas are untouched. */
mpmc_status mpmc_replica_set_state(mpmc_handle h, int32_t r, const float *xy,
                                   const uint32_t *start, uint64_t sweep, const uint32_t *tags);

/* Utility: copy accumulators acc[2N] and tags[N] to host memory (sync),
 * list order.  The accumulators measure diffusion (mean-square
 * displacement); the paper has no such observable. */
mpmc_status mpmc_get_aux(mpmc_handle h, float *acc, uint32_t *tags);
mpmc_status mpmc_replica_get_aux(mpmc_handle h, int32_t r, float *acc, uint32_t *tags);

/* Utility (state transfer): load displacement accumulators acc[2N] in the
 * list order of the current state (the order mpmc_get_aux reports), so a
 * checkpoint taken with mpmc_get_state + mpmc_get_aux resumes bit for bit
 * after mpmc_set_state (which clears them) + mpmc_set_acc (sync).
 * MPMC_EINVAL without MPMC_FLAG_ACC. */
mpmc_status mpmc_set_acc(mpmc_handle h, const float *acc);
mpmc_status mpmc_replica_set_acc(mpmc_handle h, int32_t r, const float *acc);

/* Accept bits (MPMC_FLAG_ACCEPT_LOG; Alg. 2's accept decisions): bits[c],
 * c over the cells in row-major order, has bit s set when trial s (s < 32)
 * of cell c's latest update was accepted.  A sweep updates every cell once,
 * so after a sweep this is that sweep's accept/reject sequence of every cell
 * in the grid before its shift; empty cells give 0 (sync). */
mpmc_status mpmc_get_accept_log(mpmc_handle h, uint32_t *bits);
mpmc_status mpmc_replica_get_accept_log(mpmc_handle h, int32_t r, uint32_t *bits);

/* Utility: clear the displacement accumulators of every replica (async). */
mpmc_status mpmc_reset_acc(mpmc_handle h);

/* Mean squared displacement mean(|acc|^2) over all disks, FP64, fixed
 * reduction order (sync).  Not in the paper: the diffusion figure of merit
 * of the move-size controller below. */
mpmc_status mpmc_msd(mpmc_handle h, double *msd);
mpmc_status mpmc_replica_msd(mpmc_handle h, int32_t r, double *msd);

/* Utility (invariant check: hard disks never overlap, Sec. 2.1): number of
 * ordered pairs closer than 1 - 2^-20 in r^2 in the kernels' metric, summed
 * over the replicas (sync). */
mpmc_status mpmc_count_overlaps(mpmc_handle h, int64_t *pairs);

/* Trial moves (the paper's throughput eta counts them per second, Sec. 5)
 * and accepted moves since init or the last set_state, summed
 * over the replicas (sync); the replica form gives one replica's. */
mpmc_status mpmc_get_counters(mpmc_handle h, uint64_t *trials, uint64_t *accepts);
mpmc_status mpmc_replica_get_counters(mpmc_handle h, int32_t r, uint64_t *trials,
                                      uint64_t *accepts);

/* Maximum trial displacement delta, the free parameter d of Sec. 3.3
 * (async set / sync get).  mpmc_set_delta
 * sets every replica's; the replica forms one replica's. */
mpmc_status mpmc_set_delta(mpmc_handle h, float delta);
mpmc_status mpmc_get_delta(mpmc_handle h, float *delta);
mpmc_status mpmc_replica_set_delta(mpmc_handle h, int32_t r, float delta);
mpmc_status mpmc_replica_get_delta(mpmc_handle h, int32_t r, float *delta);

/* n_M, the trial moves per active cell and sub-sweep (Alg. 1), of every
 * replica or of replica r, from the next launch on (sync: waits for the
 * stream, rewrites the replica table, re-captures the sweep graphs).  It
 * changes the chain, as delta does; 0 <= n_moves <= 2^20. */
mpmc_status mpmc_set_n_moves(mpmc_handle h, int32_t n_moves);
mpmc_status mpmc_replica_set_n_moves(mpmc_handle h, int32_t r, int32_t n_moves);

/* Plain acceptance-ratio tuner for equilibration (not in the paper, which
 * fixes d; it only sets delta before production) (async): n_windows times,
 * run window_sweeps sweeps, then with a = accepts/trials of that window
 * set delta <- delta * clamp(a/0.3, 0.5, 2), clamped to [1e-3, min(w)/2],
 * on the device, for each replica from its own counts. */
mpmc_status mpmc_tune(mpmc_handle h, int32_t window_sweeps, int32_t n_windows);

/* Utility (performance only): launch shape of the sub-sweep: lanes
 * cooperating on one active cell (1, 2
 * or 4: the group splits the neighbour cells, their filtering and the
 * overlap tests, and combines its verdicts; 64: one wavefront per cell, one
 * neighbourhood slot per lane, the verdicts combined by a wave ballot -- the
 * slow mapping, kept for comparison) and workgroup size in lanes (64, 128,
 * 192 or 256; reduced where the neighbour rows would exceed 64 KB of LDS).
 * Results do not depend on either: every comparison is the same.  The
 * launch shape applies to the separate sub-sweep launches, which the fused
 * sweep replaces unless mpmc_set_sweep_kernel(h, 0). */
mpmc_status mpmc_set_launch(mpmc_handle h, int32_t lanes_per_cell, int32_t block_size);

/* Utility (performance only): how mpmc_sweep launches a sweep.  fused != 0
 * (the default) runs each whole sweep of every replica -- the four
 * sub-sweeps in the sweep's set order, then the shift and rebuild -- as one
 * tiled launch that keeps a tile of cells with a five-cell halo in LDS and
 * recomputes the halo's updates, where that form is supported (every
 * replica of capacity 4, i.e. cells narrower than sqrt(2)); fused == 0, or
 * an unsupported handle, launches the four sub-sweeps and the rebuild
 * separately.  The chain is the same, bit for bit.  mpmc_get_sweep_kernel
 * reports whether sweeps of this handle run fused (1) or not (0).  Host
 * only. */
mpmc_status mpmc_set_sweep_kernel(mpmc_handle h, int32_t fused);
mpmc_status mpmc_get_sweep_kernel(mpmc_handle h, int32_t *fused);

/* Utility (performance only): the fused sweep's tiling.  *tile is the
 * largest tile interior side (in cells) the kernel is compiled for, which
 * depends on the buffer flags; *tx x *ty is the interior of the tile shape
 * chosen for this handle's grids and the device's compute-unit count.  All
 * three are 0 when sweeps of this handle do not run fused.  Host only. */
mpmc_status mpmc_get_fused_tile(mpmc_handle h, int32_t *tile, int32_t *tx, int32_t *ty);

/* Utility (performance only): autotuner for the launch shape.  Only shape
 * knobs that leave results bit
 * for bit unchanged are searched (lanes per cell 1, 2, 4 times workgroup
 * size 64, 128, 192, 256: twelve candidates), so the sweeps it times are
 * ordinary sweeps of the chain: for each candidate it runs `sweeps` sweeps
 * to capture and warm the graph, then times `sweeps` more with HIP events on
 * the stream, and finally keeps the fastest shape.  `sweeps` >= 16; the chain
 * advances by 2 * sweeps per candidate (24 * sweeps in all).  sync.  Any
 * output may be NULL. */
mpmc_status mpmc_autotune(mpmc_handle h, int32_t sweeps, int32_t *lanes_out, int32_t *block_out,
                          double *us_per_sweep_out);

/* Utility: every replica's counters since its init or set_state, current
 * delta and,
 * if msd is not NULL, mean |acc|^2 over its disks (FP64, fixed order), each
 * an array of R entries (sync).  Any pointer may be NULL. */
mpmc_status mpmc_batch_stats(mpmc_handle h, uint64_t *trials, uint64_t *accepts, float *delta,
                             double *msd);

/* ---- Learned move-size controller --------------------------------------
 * Not part of the paper's method: it sets the free parameter delta (Sec.
 * 3.3) between equilibration windows only, so the chain sampled afterwards
 * with delta frozen is the paper's.  The network is a 3 -> 32 -> 32 -> 1
 * perceptron with tanh hidden layers, FP32, MPMC_MLP_PARAMS parameters in
 * one device vector laid out row-major as W1[32][3] b1[32] W2[32][32] b2[32]
 * W3[1][32] b3[1].  Inputs of a replica: 20 (phi - 0.7), N/cells - 1.5 and
 * 4 (a - 0.3), with a the acceptance of the last window; output y gives
 * delta = 0.1 exp(y) clamped to [1e-3, min(w)/2].  All pointers below are
 * device pointers; the calls only enqueue work (async). */
#define MPMC_MLP_PARAMS 1217

/* Controller in the chain (async): n_windows times, run window_sweeps
 * sweeps of every replica, then set each replica's delta from the network
 * W (device, MPMC_MLP_PARAMS floats) and that window's acceptance. */
mpmc_status mpmc_control(mpmc_handle h, const float *W, int32_t window_sweeps, int32_t n_windows);

/* Utility: bytes of device workspace for mpmc_mlp_backward / mpmc_mlp_mse
 * on n samples (host only). */
mpmc_status mpmc_mlp_work_bytes(int32_t n, size_t *bytes);

/* Y[i] = net(X[i][0..2]) for n samples; X row-major [n][3].  cache, if not
 * NULL, receives the hidden activations [64][n] (feature-major) that
 * mpmc_mlp_backward needs. */
mpmc_status mpmc_mlp_forward(const float *W, const float *X, int32_t n, float *Y, float *cache,
                             void *stream);

/* Gradients of sum_i dY[i] * Y[i] with respect to the parameters (dW,
 * MPMC_MLP_PARAMS floats, overwritten) and, if dX is not NULL, the inputs
 * (dX [n][3]).  Per-workgroup partial sums are reduced in a fixed order, so
 * results do not vary from run to run.  work: mpmc_mlp_work_bytes(n). */
mpmc_status mpmc_mlp_backward(const float *W, const float *X, const float *cache, const float *dY,
                              int32_t n, float *dW, float *dX, void *work, void *stream);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): mpmc_mlp_backward with the same results, bit for bit, and the
 * same kernels, but its per-workgroup gradient rows live in a device array
 * of the library (4.6 MiB per GPU, kept until the process ends) instead of
 * a `work` argument.  Allocates nothing.  n <= MPMC_MLP_NOALLOC_MAX_SAMPLES,
 * else MPMC_EINVAL.  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other threads) race; calls in
 * order on one stream do not.  async. */
#define MPMC_MLP_NOALLOC_MAX_SAMPLES 65536
mpmc_status mpmc_mlp_backward_noalloc(const float *W, const float *X, const float *cache,
                                      const float *dY, int32_t n, float *dW, float *dX,
                                      void *stream);

/* Squared-error loss 1/(2n) sum (Y - T)^2 into *loss (device FP64) and its
 * gradient dY = (Y - T)/n.  work: mpmc_mlp_work_bytes(n). */
mpmc_status mpmc_mlp_mse(const float *Y, const float *T, int32_t n, float *dY, double *loss,
                         void *work, void *stream);

/* One Adam step (Kingma and Ba, ICLR 2015, Alg. 1) on n_params parameters:
 * m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, W <- W - lr m_hat /
 * (sqrt(v_hat) + eps) with bias corrections 1/(1 - b^step), step >= 1. */
mpmc_status mpmc_adam_step(float *W, float *m, float *v, const float *dW, int32_t n_params,
                           float lr, float b1, float b2, float eps, int32_t step, void *stream);

/* Utility: wait for all work enqueued by this handle; reports MPMC_EDEVICE
 * if a kernel set the error word. */
mpmc_status mpmc_synchronize(mpmc_handle h);

/* Utility: free the handle and its graphs (not the caller's buffers). */
void mpmc_destroy(mpmc_handle h);

/* Utility: message describing the calling thread's last failure ("" if
 * none). */
const char *mpmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPMC_H */
