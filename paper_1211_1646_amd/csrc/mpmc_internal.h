// Internal declarations shared by the host API (mpmc_api.cpp) and the
// kernels (mpmc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmc {

constexpr int kHistBins = 200;
constexpr uint32_t kErrCapacity = 1u;     // a cell holds more disks than its capacity
constexpr uint32_t kErrCount = 2u;        // rebuilt cell list does not hold N disks

// Device control block: everything a captured sweep graph reads or writes
// that changes between launches lives here, not in kernel arguments.
struct alignas(256) Ctl {
    unsigned long long sweep;        // current sweep index s
    unsigned long long trials;       // trial moves since init / set_state
    unsigned long long accepts;      // accepted moves
    unsigned long long win_trials;   // counters at the start of the tuner window
    unsigned long long win_accepts;
    unsigned int key0, key1;         // Philox key (seed, replica)
    float delta;                     // maximum trial displacement
    unsigned int errword;            // kErr* bits set by kernels
    unsigned int pad0[2];
    // Sweep-global draws of sweep s in draw[s & 1]: set order (byte q = set
    // of slot q), shift direction f and distance d.  Written when the sweep
    // counter or the key changes, read by every launch of the sweep.
    struct Draw {
        unsigned int order;
        int f;
        float d;
        unsigned int pad;
    } draw[2];
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

// Per-sweep draws shared by the sub-sweep and rebin launches.
struct SweepBuffers {
    const float2 *pos;
    const uint32_t *start;
    const float2 *acc;
    const uint32_t *tag;
};

// Scratch layout (caller's work buffer): u32 scan partials of the rebin,
// then per-workgroup trial/accept partials (slot-major [slot][trials|accepts]
// [tile]: slots 0-3 are the four sub-sweeps of a sweep, slot 4 accumulates
// lone sub-sweeps), then FP64 reduction partials.
struct Work {
    uint32_t *scan;    // scan_partials(C) entries
    uint32_t *cnt;     // 10 * count_stride(C) entries
    double *f64;       // kMsdBlocksMax entries
    int cnt_stride;
};

// ---- launch wrappers (defined in mpmc_kernels.hip) ----
// Sub-sweep of one checkerboard set; set >= 0 explicit (its counters go to
// the lone slot, folded by launch_fold_lone), set < 0 means the sweep's slot
// (-1 - set) of the shuffled set order (counters folded by the rebin).  The
// workgroup size is at most 256 (LDS: 8 * cap float2 per lane).
hipError_t launch_subsweep(const Geom &g, float2 *pos, const uint32_t *start, float2 *acc,
                           uint32_t *tag, Ctl *ctl, const Work &w, int n_moves, int set,
                           int lanes_per_cell, int block, hipStream_t st);

// Shift (f, d) -- or the sweep's own draws when f < 0 -- and rebuild the
// cell lists into the *_out buffers.  advance != 0 increments the sweep.
hipError_t launch_fold_lone(const Work &w, Ctl *ctl, hipStream_t st);

// With f < 0 it also folds the four sub-sweeps' counters (sub_block = their
// workgroup size) into the control block.
hipError_t launch_rebin(const Geom &g, const float2 *pos, const uint32_t *start,
                        const float2 *acc, const uint32_t *tag, float2 *pos_out,
                        uint32_t *start_out, float2 *acc_out, uint32_t *tag_out,
                        const Work &w, Ctl *ctl, int f, float d, int advance, int block,
                        int sub_block, hipStream_t st);

hipError_t launch_pair_histogram(const Geom &g, const float2 *pos, const uint32_t *start,
                                 Ctl *ctl, int reset, int block, hipStream_t st);
hipError_t launch_pressure_fit(const Geom &g, Ctl *ctl, hipStream_t st);
hipError_t launch_count_overlaps(const Geom &g, const float2 *pos, const uint32_t *start,
                                 Ctl *ctl, int block, hipStream_t st);
hipError_t launch_msd(const Geom &g, const float2 *acc, const Work &w, Ctl *ctl,
                      hipStream_t st);
// apply == 0 only opens a new tuner window (records the counters).
hipError_t launch_tune(const Geom &g, Ctl *ctl, int apply, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, long long n, hipStream_t st);
hipError_t launch_ctl_reset(const Geom &g, Ctl *ctl, unsigned long long sweep, unsigned int key0,
                            unsigned int key1, float delta, hipStream_t st);
hipError_t launch_ctl_set_key0(const Geom &g, Ctl *ctl, unsigned int key0, hipStream_t st);
hipError_t launch_ctl_set_delta(Ctl *ctl, float delta, hipStream_t st);

// Work-buffer sizes, from the smallest workgroup allowed.
constexpr int kMinBlock = 64;
constexpr int kMsdBlocksMax = 512;
inline long long scan_partials(long long C) { return (C + kMinBlock - 1) / kMinBlock + 8; }
inline long long count_stride(long long C) { return (C / 4 + kMinBlock - 1) / kMinBlock + 8; }

}  // namespace mpmc
