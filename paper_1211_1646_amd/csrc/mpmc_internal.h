// Internal declarations shared by the host API (mpmc_api.cpp) and the
// kernels (mpmc_kernels.hip).  Not part of the public ABI.
//
// Every handle holds R >= 1 independent systems ("replicas").  Their cells and
// disks are concatenated in one compressed-row layout; each replica's cell
// range is padded to whole rebin tiles and its active-cell range to whole
// active chunks, so that every workgroup of every kernel belongs to exactly
// one replica and finds it with one table load.  A single system is the
// batch with R = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmc {

constexpr int kHistBins = 200;
constexpr uint32_t kErrCapacity = 1u;     // a cell holds more disks than its capacity
constexpr uint32_t kErrCount = 2u;        // rebuilt cell list does not hold N disks

constexpr int kRebinTile = 256;           // cells per rebin workgroup (one per thread)
constexpr int kActiveChunk = 768;         // active-slot granularity (lcm of 64, 128, 192, 256)
constexpr int kGranule = 64;              // counter partials: one per 64 active slots
constexpr int kMsdBlocksMax = 512;
constexpr int kMlpParams = 1217;          // 3 -> 32 -> 32 -> 1 network
constexpr int kNbrLds = 16;               // reachable neighbours a lane keeps in LDS
constexpr int kAblateParticleShuffle = 1; // Rep::ablate: visit cells in stored order
constexpr int kAblateSetShuffle = 2;      // Rep::ablate: sets always a, b, c, d
constexpr int kAblateLeave = 4;           // Rep::ablate: moves may leave the cell by (w - 1)/2
constexpr int kAblateLeaveOnce = 8;       // Rep::ablate: as kAblateLeave, n_M = n

// Per-replica control block: everything a captured sweep graph reads or
// writes that changes between launches lives here, not in kernel arguments.
struct alignas(256) Ctl {
    // Current sweep index s, by buffer parity: a launch that reads ping-pong
    // half p reads sweep_at[p] and draw_at[p]; the rebin, which reads half p
    // and writes half p ^ 1, writes slot p ^ 1 (s + 1 and its draws, or a
    // copy for an explicit shift), so no launch writes what it reads.
    unsigned long long sweep_at[2];
    unsigned long long trials;       // trial moves since init / set_state (folded)
    unsigned long long accepts;      // accepted moves (folded)
    unsigned long long win_trials;   // counters at the start of the tuner window
    unsigned long long win_accepts;
    unsigned int key0, key1;         // Philox key (seed, replica)
    float delta;                     // maximum trial displacement
    unsigned int errword;            // kErr* bits set by kernels
    // Sweep-global draws of sweep_at[p]: set order (byte q = set of slot q),
    // shift direction f and distance d.  Rewritten when the key changes.
    struct Draw {
        unsigned int order;
        int f;
        float d;
        unsigned int pad;
    } draw_at[2];
    unsigned long long hist_samples; // configurations in hist[]
    double fit[4];                   // P*, g(sigma+), rho, status
    long long overlaps;              // ordered overlapping pairs (count kernel)
    double msd;                      // mean |acc|^2
    unsigned long long hist[kHistBins];
};

struct Geom {
    int mx, my, C, cap;
    float wx, wy;
    long long N;
};

// Placement and initial parameters of one replica.
struct Rep {
    Geom g;
    long long cb;        // first global cell; multiple of kRebinTile
    long long cpad;      // padded cell count; multiple of kRebinTile
    long long pb;        // first global disk
    long long ab;        // first global active slot; multiple of kActiveChunk
    long long apad;      // padded active-slot count; multiple of kActiveChunk
    int n_moves;
    unsigned int key0, key1;
    float delta0;
    int disk;            // 1: in-circle trial moves, 0: square
    int ablate;          // kAblate* bits: shuffles switched off (Table 1)
    int tiles_x, tiles_y; // tiles of the fused sweep over this replica's grid
    long long tb;        // the replica's first fused-sweep tile
};

// Device tables of a handle (in the caller's control buffer), passed to the
// kernels by value.
struct Tables {
    Rep rep0;               // replica 0 by value: a single system needs no table load
    const Rep *reps;        // [R]
    Ctl *ctls;              // [R]
    const uint16_t *arep;   // replica of each active chunk
    const uint16_t *crep;   // replica of each rebin tile
    const uint16_t *trep;   // replica of each fused-sweep tile
    long long ftiles;       // fused-sweep tiles, all replicas
    int ftile;              // largest fused-sweep tile side (cells), set by the buffer flags
    int ftx, fty;           // the tile shape in use (cells, even, at most ftile)
    int R;
    int cap;                // largest capacity
    int prop;               // sub-sweep variant: 0 all square, 1 all in-circle, 2 per replica
                            // (mixed proposals, the particle-shuffle or leaving pitfalls)
    int leave;              // some replica lets disks leave their cells (general rebuild)
    long long cells;        // padded cells, all replicas
    long long active;       // padded active slots, all replicas
    long long N;            // disks, all replicas
};

// Scratch (caller's work buffer): u64 trial/accept partials per granule of
// active slots (accumulated by every sub-sweep, folded into the control
// blocks on demand), FP64 partials, and per active slot the reachable
// neighbours beyond the first kNbrLds.
struct Work {
    unsigned long long *cnt;     // [2][cnt_stride]
    double *f64;                 // kMsdBlocksMax entries
    float2 *ovf;                 // [active][ovf_per_slot(cap)]
    int cnt_stride;
};

inline long long count_stride(long long active) { return active / kGranule + 8; }
inline int ovf_per_slot(int cap) { return 8 * cap > kNbrLds ? 8 * cap - kNbrLds : 0; }

// ---- launch wrappers (defined in mpmc_kernels.hip) ----
// Sub-sweep of every replica; set >= 0 is the same explicit set everywhere,
// set < 0 is each replica's slot (-1 - set) of its own shuffled set order.
// lanes (1, 2 or 4) lanes work on each active cell; the workgroup size is
// 64, 128, 192 or 256 lanes (reduced if the LDS rows would not fit).
// alog (may be null): per-cell accept bits of this launch's active cells.
// par: the ping-pong half being read (selects the sweep slot).
hipError_t launch_subsweep(const Tables &t, int par, float2 *pos, const uint32_t *count,
                           float2 *acc, uint32_t *tag, uint32_t *alog, const Work &w, int set,
                           int block, int lanes, hipStream_t st);
// Add the counter partials into each replica's control block; clear them.
hipError_t launch_fold_counters(const Tables &t, const Work &w, hipStream_t st);
// Shift (f, d) -- or each replica's own draws when f < 0 -- and rebuild the
// cell lists into the *_out buffers (half par ^ 1); advance moves every
// replica on to its next sweep (only with f < 0).
hipError_t launch_rebin(const Tables &t, int par, const float2 *pos, const uint32_t *count,
                        const float2 *acc, const uint32_t *tag, float2 *pos_out,
                        uint32_t *count_out, float2 *acc_out, uint32_t *tag_out,
                        const Work &w, int f, float d, int advance, hipStream_t st);
// A whole sweep (the four sub-sweeps in the sweep's set order, then the
// shift and rebuild with the sweep's own draws) of every replica in one
// launch: reads half par, writes half par ^ 1 and advances every replica's
// sweep.  The same chain as launch_subsweep x 4 + launch_rebin, bit for bit.
// Supported when every replica has capacity 4 (slot layout of 4).
// fused_tile: the largest tile side the handle's buffer flags allow (LDS
// for two workgroups per CU); the shape in use is chosen per handle.
constexpr int kFusedMinTile = 16;
int fused_tile(bool acc, bool tag);
bool sweep_fused_supported(const Tables &t);
hipError_t launch_sweep_fused(const Tables &t, int par, const float2 *pos, const uint32_t *count,
                              const float2 *acc, const uint32_t *tag, float2 *pos_out,
                              uint32_t *count_out, float2 *acc_out, uint32_t *tag_out,
                              uint32_t *alog, const Work &w, hipStream_t st);
hipError_t launch_pair_histogram(const Tables &t, const float2 *pos, const uint32_t *count,
                                 int reset, hipStream_t st);
hipError_t launch_pressure_fit(const Tables &t, int replica, hipStream_t st);
hipError_t launch_count_overlaps(const Tables &t, const float2 *pos, const uint32_t *count,
                                 hipStream_t st);
// Mean |acc|^2 over the N disks of one replica into its control block.
hipError_t launch_msd(const Tables &t, int replica, long long N, const float2 *acc,
                      const uint32_t *count, const Work &w, hipStream_t st);
// apply == 0 only opens a new tuner window (records the counters); call after
// launch_fold_counters.
hipError_t launch_tune(const Tables &t, int apply, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, long long n, hipStream_t st);
// Reset the control block of replica r (every replica when r < 0) to sweep,
// its initial key and delta.
hipError_t launch_ctl_reset(const Tables &t, int replica, unsigned long long sweep,
                            hipStream_t st);
hipError_t launch_ctl_set_key0(const Tables &t, unsigned int key0, hipStream_t st);
hipError_t launch_ctl_set_delta(const Tables &t, int replica, float delta, hipStream_t st);
// Workgroup size the sub-sweep actually uses for a requested one.
int subsweep_block(int cap, int block, int lanes);
// Mean |acc|^2 of every replica into its control block (one workgroup each).
hipError_t launch_msd_all(const Tables &t, const float2 *acc, const uint32_t *count, hipStream_t st);

// ---- move-size network (defined in mpmc_mlp.hip) ----
size_t mlp_work_bytes(int n);
hipError_t launch_mlp_forward(const float *W, const float *X, int n, float *Y, float *cache,
                              hipStream_t st);
hipError_t launch_mlp_backward(const float *W, const float *X, const float *cache,
                               const float *dY, int n, float *dW, float *dX, void *work,
                               hipStream_t st);
// The same backward pass with its gradient rows in the library's own device
// array (no workspace argument, nothing allocated); n <= 65536.
hipError_t launch_mlp_backward_noalloc(const float *W, const float *X, const float *cache,
                                       const float *dY, int n, float *dW, float *dX,
                                       hipStream_t st);
hipError_t launch_mse(const float *Y, const float *T, int n, float *dY, double *loss, void *work,
                      hipStream_t st);
hipError_t launch_adam(float *W, float *m, float *v, const float *g, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st);
// Controller step of every replica from its window counters (apply == 0
// only opens a window); call after launch_fold_counters.
hipError_t launch_control(const Tables &t, const float *W, int apply, hipStream_t st);

}  // namespace mpmc
