// Internal declarations shared by the host side (sphere_api.cpp) and the
// kernels (sphere_kernels.hip) of the 3D hard-sphere chain.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmc {
namespace sph {

constexpr int kCap = 8;                  // spheres per cell (w < 2/sqrt(3))
constexpr int kPrim = 2;                 // slots in a cell's primary line
constexpr int kHistBins = 200;
constexpr uint32_t kErrCapacity = 1u;    // a cell holds more than kCap spheres
constexpr int kTile = 256;               // cells per rebin / histogram workgroup
constexpr int kSubBlock = 64;            // lanes per sub-sweep workgroup (one wave)
constexpr int kNbrList = 32;             // reachable neighbours a lane keeps in LDS

// Control block: what a captured sweep graph reads or writes that changes
// between launches.  sweep_at / draw_at are indexed by the ping-pong half a
// launch reads; the rebin, which reads half p and writes p ^ 1, writes slot
// p ^ 1, so no launch writes what it reads.
struct alignas(256) Ctl3 {
    unsigned long long sweep_at[2];
    unsigned long long trials, accepts;   // folded counters
    unsigned long long win_trials;        // counters at the start of the tuner window
    unsigned long long win_accepts;
    unsigned int key0, key1;
    float delta;
    unsigned int errword;
    struct Draw {
        unsigned int order;   // nibble q = set processed in slot q
        int f;                // 0..5 = +x, -x, +y, -y, +z, -z
        float d;
        unsigned int pad;
    } draw_at[2];
    unsigned long long hist_samples;
    double fit[4];                        // P, g(sigma+), rho, status
    long long overlaps;
    double msd;                           // mean |acc|^2
    unsigned long long hist[kHistBins];
};

struct Geom3 {
    int m[3];        // cells per axis (even, >= 4)
    float w[3];      // cell widths
    int C;           // cells
    int active;      // active cells of one set: C / 8
    long long N;
    int n_moves;
};

// Slot i of cell c among the C cells' slots: slots 0..1 sit in the cell's
// 32-byte primary line (2 c + i), slots 2..7 -- needed only by the cells
// with more than two spheres, about one in ten at eta = 0.45 -- in an
// overflow region after every primary line (2 C + 6 c + i - 2).  A cell's
// usual spheres then share one 32-byte sector instead of a 128-byte line of
// eight slots.
__host__ __device__ inline size_t slot_of(int C, int c, int i)
{
    return i < kPrim ? (size_t)c * kPrim + (size_t)i
                     : (size_t)kPrim * (size_t)C + (size_t)c * (kCap - kPrim) + (size_t)(i - kPrim);
}

// Sub-sweep workgroups for `lanes` (1, 2 or 4) lanes per active cell, and
// the counter partials: two u64 (trials, accepts) per workgroup of the
// widest launch, accumulated by every sub-sweep and folded on demand.
inline int subsweep_tiles(const Geom3 &g, int lanes)
{
    return (int)(((long long)g.active * lanes + kSubBlock - 1) / kSubBlock);
}
// Bricks of 4 x 4 x 4 active cells along an axis of m cells (m / 2 active),
// for the one-lane form; the partials cover whichever launch has more groups.
inline int brick_count(int m) { return (m / 2 + 3) / 4; }
inline int subsweep_groups(const Geom3 &g)
{
    const int bricks = brick_count(g.m[0]) * brick_count(g.m[1]) * brick_count(g.m[2]);
    const int tiles = subsweep_tiles(g, 4);
    return bricks > tiles ? bricks : tiles;
}
inline int xcd_groups(int tiles) { return 8 * ((tiles + 7) / 8); }

hipError_t launch_subsweep3(const Geom3 &g, Ctl3 *ctl, int par, float4 *pos,
                            const uint32_t *count, uint32_t *tag, float4 *acc,
                            unsigned long long *cnt, int set, int lanes, hipStream_t st);
hipError_t launch_fold3(const Geom3 &g, Ctl3 *ctl, unsigned long long *cnt, hipStream_t st);
// f >= 0: explicit shift (f, d), sweep slot copied; f < 0: the sweep's own
// draws, advance to the next sweep.
hipError_t launch_rebin3(const Geom3 &g, Ctl3 *ctl, int par, const float4 *pos,
                         const uint32_t *count, const uint32_t *tag, const float4 *acc,
                         float4 *pos_out, uint32_t *count_out, uint32_t *tag_out, float4 *acc_out,
                         int f, float d, hipStream_t st);
// Mean |acc|^2 over the spheres into ctl->msd (FP64, fixed order); part
// holds ceil(C / kTile) doubles.
hipError_t launch_msd3(const Geom3 &g, Ctl3 *ctl, const float4 *acc, const uint32_t *count,
                       double *part, hipStream_t st);
hipError_t launch_zero4(float4 *p, long long n, hipStream_t st);
hipError_t launch_ctl_reset3(const Geom3 &g, Ctl3 *ctl, unsigned long long sweep,
                             unsigned int key0, unsigned int key1, float delta, hipStream_t st);
hipError_t launch_set_delta3(Ctl3 *ctl, float delta, hipStream_t st);
// Plain acceptance tuner: apply == 0 only opens a window (records the
// counters); call after launch_fold3.
hipError_t launch_tune3(const Geom3 &g, Ctl3 *ctl, int apply, hipStream_t st);
hipError_t launch_pair_hist3(const Geom3 &g, Ctl3 *ctl, const float4 *pos, const uint32_t *count,
                             int reset, hipStream_t st);
hipError_t launch_pressure_fit3(const Geom3 &g, Ctl3 *ctl, hipStream_t st);
hipError_t launch_count_overlaps3(const Geom3 &g, Ctl3 *ctl, const float4 *pos,
                                  const uint32_t *count, hipStream_t st);

}  // namespace sph

// Record the calling thread's failure message (read by mpmc_last_error).
void set_last_error(const char *msg);

}  // namespace mpmc
