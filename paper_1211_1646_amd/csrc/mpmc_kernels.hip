// HIP kernels of the MPMC hard-disk sweep for gfx950 (CDNA4, wave64).
//
// Method: Anderson et al., "Massively parallel Monte Carlo for many-particle
// simulations on GPUs" -- Alg. 1 (sweep), Alg. 2 (sub-sweep), Alg. 4 (cell
// shift), Sec. 4 (contact-value pressure, Eqs. gR, R, P).
//
// Data layout in device memory (the paper's disk[x, y, i], Sec. 3.1):
//   count[C]      uint32 disks per cell, cells in row-major order;
//   pos[C][CAP]   float2 cell-local coordinates in (0, w], slots [0, count)
//                 used, CAP = the largest capacity of the handle's replicas;
//   acc[C][CAP]   float2 displacement accumulators (optional), tag[C][CAP]
//                 (optional), in the same slots.
// Fixed slots let a kernel load a cell's count and its disks together, in
// one memory round trip, and let the rebin write each new cell without a
// scan.  A sub-sweep writes only the active cells' own slots and reads the
// eight inactive neighbours, so it updates in place; the rebin writes the
// other ping-pong half.
//
// Every floating-point expression is written so that each operation rounds
// once (no contraction); the library is built with -ffp-contract=off and the
// pragma below repeats it for these kernels.
#include <utility>

#include "mpmc_device.h"
#include "mpmc_internal.h"

#pragma clang fp contract(off)

namespace mpmc {
namespace {

constexpr uint32_t kTagShuffle = 0x40000000u;
constexpr uint32_t kTagSweep = 0x80000000u;
constexpr uint32_t kCellGlobal = 0xFFFFFFFFu;

// Trial displacement from one word: high half -> x, low half -> y, each the
// midpoint (2h + 1 - 65536) / 65536 of a sub-interval of (-1, 1), times delta.
__device__ __forceinline__ void displacement(uint32_t u, float delta, float &dx, float &dy)
{
    const int hx = (int)(u >> 16);
    const int hy = (int)(u & 0xFFFFu);
    const float ux = (float)(2 * hx + 1 - 65536) * 0x1p-16f;
    const float uy = (float)(2 * hy + 1 - 65536) * 0x1p-16f;
    dx = ux * delta;
    dy = uy * delta;
}

// In-circle trial displacement (Alg. 2's inCircle(d)) from one word.
//   radius: sqrt of the midpoint (2 hr + 1) / 2^17 of one of 65536 equal parts
//           of (0, 1) -- uniform in area -- times delta;
//   angle:  (2 ha + 1) pi / 65536; bits 15..14 of ha are the quarter turn,
//           bits 13..0 the angle inside the quarter.  Angles above pi/4 use
//           the mirror angle below it with cos and sin exchanged, so the
//           series only see (0, pi/4): Taylor to x^9 (sin) and x^10 (cos),
//           remainders below 2e-9.
// Every operation is a single FP32 operation in the order written
// (contraction is off; sqrtf is the correctly rounded square root), and a
// quarter turn only permutes and negates, so words differing in bit 15 give
// exactly opposite moves.
__device__ __forceinline__ void disk_displacement(uint32_t u, float delta, float &dx, float &dy)
{
    const uint32_t ha = u & 0xFFFFu;
    const uint32_t jq = ha & 0x3FFFu;
    const bool upper = jq >= 8192u;
    const uint32_t m = upper ? 16383u - jq : jq;
    const float x = (float)(2u * m + 1u) * 0x1.921fb6p-15f;     // pi / 65536
    const float z = x * x;
    float ps = 0x1.71de3ap-19f * z;                              // 1/9!
    ps = ps + -0x1.a01a02p-13f;                                  // -1/7!
    ps = ps * z;
    ps = ps + 0x1.111112p-7f;                                    // 1/5!
    ps = ps * z;
    ps = ps + -0x1.555556p-3f;                                   // -1/3!
    const float sn = x + (x * z) * ps;
    float pc = -0x1.27e4fcp-22f * z;                             // -1/10!
    pc = pc + 0x1.a01a02p-16f;                                   // 1/8!
    pc = pc * z;
    pc = pc + -0x1.6c16c2p-10f;                                  // -1/6!
    pc = pc * z;
    pc = pc + 0x1.555556p-5f;                                    // 1/4!
    pc = pc * z;
    pc = pc + -0.5f;                                             // -1/2!
    const float cs = 1.0f + z * pc;
    const float c = upper ? sn : cs;
    const float sv = upper ? cs : sn;
    // quarter turns: (c, s) -> (-s, c) -> (-c, -s) -> (s, -c)
    const uint32_t q = ha >> 14;
    const float a0 = (q & 1u) ? sv : c;
    const float b0 = (q & 1u) ? c : sv;
    const float a = ((q + 1u) & 2u) ? -a0 : a0;
    const float b = (q & 2u) ? -b0 : b0;
    const float r = __builtin_sqrtf((float)(2u * (u >> 16) + 1u) * 0x1p-17f) * delta;
    dx = r * a;
    dy = r * b;
}

struct Draws {
    uint32_t order;   // byte q = set processed in slot q
    int f;
    float d;
};

// The sweep-global block (Alg. 1): Fisher-Yates order of
// the four sets from words 0..2; f from the top two bits of word 3 and
// d = u (w_f / 2) from its low 24 bits.  The order is kept as four bytes of
// one register so that no array is indexed at run time.
__device__ __forceinline__ Draws sweep_draws(unsigned long long s, uint32_t k0, uint32_t k1,
                                             float wx, float wy, bool shuffle_sets)
{
    const uint4 G = philox(kCellGlobal, (uint32_t)s, (uint32_t)(s >> 32), kTagSweep, k0, k1);
    Draws D;
    uint32_t ord = 0x03020100u;
#pragma unroll
    for (int i = 3; i >= 1; --i) {
        if (!shuffle_sets) break;   // the set-shuffle ablation (Table 1): a, b, c, d
        const uint32_t j = bounded(word_of(G, 3 - i), (uint32_t)(i + 1));
        const uint32_t oi = (ord >> (8 * i)) & 0xFFu;
        const uint32_t oj = (ord >> (8 * j)) & 0xFFu;
        ord = (ord & ~(0xFFu << (8 * i))) | (oj << (8 * i));
        ord = (ord & ~(0xFFu << (8 * j))) | (oi << (8 * j));
    }
    D.order = ord;
    D.f = (int)(G.w >> 30);
    const float w = D.f < 2 ? wx : wy;
    const float u = (float)(G.w & 0xFFFFFFu) * 0x1p-24f;
    D.d = u * (0.5f * w);
    return D;
}

// Record sweep s and its draws in sweep slot p of the control block (one
// thread).
__device__ __forceinline__ void store_draws(Ctl *ctl, int p, unsigned long long s, const Rep &R)
{
    const Draws D = sweep_draws(s, ctl->key0, ctl->key1, R.g.wx, R.g.wy,
                                (R.ablate & kAblateSetShuffle) == 0);
    ctl->sweep_at[p] = s;
    Ctl::Draw &r = ctl->draw_at[p];
    r.order = D.order;
    r.f = D.f;
    r.d = D.d;
}

// Replica of a workgroup and its table entry.  With one replica both are
// known from the kernel arguments, which saves two dependent loads.
__device__ __forceinline__ int chunk_replica(const Tables &t, bool in, long long chunk)
{
    return (t.R == 1 || !in) ? 0 : (int)t.arep[chunk];
}
__device__ __forceinline__ int tile_replica(const Tables &t, bool in, int tile)
{
    return (t.R == 1 || !in) ? 0 : (int)t.crep[tile];
}
__device__ __forceinline__ Rep rep_of(const Tables &t, int r) { return t.R == 1 ? t.rep0 : t.reps[r]; }

// Sum of one value per thread over the workgroup (blockDim <= 1024).
__device__ __forceinline__ unsigned block_sum_u32(unsigned v, unsigned *scratch16)
{
    v = wave_sum_u32(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch16[wave] = v;
    __syncthreads();
    unsigned total = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) total += scratch16[q];
    __syncthreads();
    return total;
}

// ------------------------------------------------------------ sub-sweep
// One lane per active cell of set Q (Alg. 2).  Disks live in fixed slots,
// CAP per cell (the paper's disk[x, y, i], Sec. 3.1), so the kernel exposes
// memory-level parallelism rather than chasing pointers:
//   1-2. the nine counts of the 3x3 block and all its 9 CAP slots are loaded
//      at once, in one memory round trip (slots past a count hold stale
//      values and are masked afterwards); the Philox blocks of the cell are
//      computed while the loads fly;
//   3. neighbour disks are translated into the cell's frame (exactly -w, 0
//      or +w, Sec. 3.1) and those that can reach the cell at all -- closer
//      than 1.0001 to the cell rectangle, a superset of every disk a trial
//      position inside the cell can overlap -- are compacted into this
//      lane's row of an LDS table (lane-major, odd row stride, so sixteen
//      lanes reading entry k hit sixteen distinct bank pairs);
//   4. the n_M trials run from registers (own cell) and LDS (neighbours).
// Dropping unreachable disks cannot change a decision: a trial outside the
// cell is rejected before any overlap test, and one inside it is at distance
// >= 1 from every dropped disk.
constexpr float kReach2 = 1.0001f;
constexpr float kReachEdge = 1.0001f;

// Neighbour disk p of the cell in row ra, column cb (0, 1, 2 = -1, 0, +1) of
// the 3x3 block, translated into the centre cell's frame by exactly -w, 0 or
// +w (adding 0 is skipped: x + 0 == x for x > 0), and whether it can reach
// the centre cell: one comparison for an edge cell, the distance to the
// shared corner for a corner cell.
__device__ __forceinline__ float2 frame_of(float2 p, int ra, int cb, float wx, float wy,
                                           bool &reach)
{
    float ox = p.x, oy = p.y;
    if (cb == 0) ox = ox - wx;
    if (cb == 2) ox = ox + wx;
    if (ra == 0) oy = oy - wy;
    if (ra == 2) oy = oy + wy;
    if (ra == 1) reach = cb == 0 ? ox > -kReachEdge : ox < wx + kReachEdge;
    else if (cb == 1) reach = ra == 0 ? oy > -kReachEdge : oy < wy + kReachEdge;
    else {
        const float ex = cb == 0 ? -ox : ox - wx;
        const float ey = ra == 0 ? -oy : oy - wy;
        reach = ex * ex + ey * ey < kReach2;
    }
    return make_float2(ox, oy);
}

// Smallest r^2 from (xm, ym) to four neighbour entries; any r^2 < 1 iff the
// smallest is (all values finite).
__device__ __forceinline__ float min_r2(float xm, float ym, const float2 *e)
{
    const float2 e0 = e[0], e1 = e[1], e2 = e[2], e3 = e[3];
    const float d0x = xm - e0.x, d0y = ym - e0.y;
    const float d1x = xm - e1.x, d1y = ym - e1.y;
    const float d2x = xm - e2.x, d2y = ym - e2.y;
    const float d3x = xm - e3.x, d3y = ym - e3.y;
    return fminf(fminf(pair_r2(d0x, d0y), pair_r2(d1x, d1y)), fminf(pair_r2(d2x, d2y), pair_r2(d3x, d3y)));
}

template <int CAP, int PROP, bool ONE>
__global__ void __launch_bounds__(256)
k_subsweep(Tables t, int par, float2 *__restrict__ pos, const uint32_t *__restrict__ count,
           float2 *__restrict__ acc, uint32_t *__restrict__ tag, uint32_t *__restrict__ alog,
           unsigned long long *__restrict__ cnt, int cnt_stride, float2 *__restrict__ ovf_all,
           int set, int ntile, int per)
{
    extern __shared__ float2 lds[];   // [blockDim.x][kRow]; reused for the counts
    // The first kL reachable neighbours of a lane live in its LDS row (odd
    // stride: 16 lanes hit distinct bank pairs); the rare rest, up to 8 CAP
    // in all, in the lane's own overflow entries in global memory.  A small
    // row keeps the LDS per workgroup low enough for four waves per SIMD.
    constexpr int kL = 8 * CAP < kNbrLds ? 8 * CAP : kNbrLds;
    constexpr int kO = 8 * CAP - kL;
    constexpr int kRow = kL + 1;
    const int tile = xcd_tile(per);
    const long long slot0 = (long long)tile * blockDim.x;
    // ONE: a single system, whose table entry is a kernel argument (read
    // with the other arguments, no dependent load)
    const int r = ONE ? 0 : chunk_replica(t, tile < ntile, slot0 / kActiveChunk);
    const Rep R = ONE ? t.rep0 : t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = t.ctls + r;
    const unsigned long long s = ctl->sweep_at[par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const int n_moves = R.n_moves;
    // proposal: fixed for the launch (PROP 0 square, 1 in-circle) or per
    // replica (PROP 2, which also carries the particle-shuffle ablation)
    const bool disk = PROP == 2 ? R.disk != 0 : PROP == 1;
    const bool shuffle = PROP == 2 ? (R.ablate & kAblateParticleShuffle) == 0 : true;
    // the cell-leaving pitfalls (Sec. 2.4, diagnostic): the trial window is
    // the cell grown by (w - 1)/2 per axis, no reach filter (neighbours may
    // sit outside their cells), and under leave-once n_M = n
    const bool leave = PROP == 2 && (R.ablate & (kAblateLeave | kAblateLeaveOnce)) != 0;
    const bool leave_once = PROP == 2 && (R.ablate & kAblateLeaveOnce) != 0;
    const float ex = leave ? (g.wx - 1.0f) * 0.5f : 0.0f;
    const float ey = leave ? (g.wy - 1.0f) * 0.5f : 0.0f;
    const float lox = -ex, hix = g.wx + ex, loy = -ey, hiy = g.wy + ey;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);

    int Q = set;
    if (Q < 0) Q = (int)((ctl->draw_at[par].order >> (8 * (-1 - set))) & 0xFFu);
    const int qx = Q & 1, qy = Q >> 1;
    const int hx = g.mx >> 1, hy = g.my >> 1;
    const int gid = (int)(slot0 - R.ab) + (int)threadIdx.x;        // within the replica
    float2 *const nbr = lds + threadIdx.x * kRow;   // this lane's neighbour list
    float2 *const ovf = ovf_all + (size_t)(slot0 + (long long)threadIdx.x) * kO;
    const uint32_t *const cn = count + R.cb;        // this replica's cell counts
    const size_t sb = (size_t)R.cb * CAP;           // and its first slot

    unsigned n_trials = 0, n_acc = 0;
    uint32_t abits = 0;
    long long log_cell = -1;   // global cell index of this lane's cell, if any
    if (tile < ntile && gid < hx * hy) {
        const int iy = (int)((unsigned)gid / (unsigned)hx), ix = gid - iy * hx;
        const int cx = 2 * ix + qx, cy = 2 * iy + qy;
        const int c = cy * g.mx + cx;
        log_cell = R.cb + c;
        const int xl = cx == 0 ? g.mx - 1 : cx - 1;
        const int xr = cx == g.mx - 1 ? 0 : cx + 1;
        const int yd = cy == 0 ? g.my - 1 : cy - 1;
        const int yu = cy == g.my - 1 ? 0 : cy + 1;
        // 1-2. counts and slots of the nine cells q = 3*row + col (row/col
        // 0, 1, 2 = -1, 0, +1), all in flight together
        uint32_t rn[9];
        float2 nv[9][CAP];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int row = q / 3 == 0 ? yd : (q / 3 == 1 ? cy : yu);
            const int col = q % 3 == 0 ? xl : (q % 3 == 1 ? cx : xr);
            const int cc = row * g.mx + col;
            rn[q] = cn[cc];
#pragma unroll
            for (int i = 0; i < CAP; ++i) nv[q][i] = pos[sb + (size_t)cc * CAP + (size_t)i];
        }
        // the cell's first shuffle block and first trial block, computed
        // while the loads are outstanding
        uint4 Wsh = make_uint4(0, 0, 0, 0);
        if (shuffle) Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle, k0, k1);
        uint4 W = make_uint4(0, 0, 0, 0);
        if (n_moves > 0 || leave_once) W = philox((uint32_t)c, s_lo, s_hi, 0u, k0, k1);
        bool bad = false;
#pragma unroll
        for (int q = 0; q < 9; ++q) bad |= rn[q] > (uint32_t)g.cap;
        int n = (int)rn[4];
        if (bad) {
            atomicOr((unsigned int *)&ctl->errword, kErrCapacity);
            n = 0;
        }
        if (n > 0) {
            const size_t b0 = sb + (size_t)c * CAP;   // own slots
            const bool has_acc = acc != nullptr, has_tag = tag != nullptr;
            float px[CAP], py[CAP], ax[CAP], ay[CAP];
            uint32_t tg[CAP];
#pragma unroll
            for (int q = 0; q < CAP; ++q) {
                px[q] = nv[4][q].x;
                py[q] = nv[4][q].y;
                ax[q] = ay[q] = 0.0f;
                tg[q] = 0u;
            }
            if (has_acc) {
#pragma unroll
                for (int q = 0; q < CAP; ++q) {
                    const float2 a = acc[b0 + (size_t)q];
                    ax[q] = a.x;
                    ay[q] = a.y;
                }
            }
            if (has_tag) {
#pragma unroll
                for (int q = 0; q < CAP; ++q) tg[q] = tag[b0 + (size_t)q];
            }
            // 3. translate into the cell's frame, keep the disks that can
            // reach the cell, compact them into the lane's LDS row.  The
            // common path has no branch: an index past kL lands on the row's
            // pad slot kL, which is never read; a lane with more than kL
            // reachable neighbours writes the rest to its overflow entries in
            // a second pass, taken only where needed.
            int K = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                if (q == 4) continue;
#pragma unroll
                for (int i = 0; i < CAP; ++i) {
                    bool reach;
                    const float2 v = frame_of(nv[q][i], q / 3, q % 3, g.wx, g.wy, reach);
                    nbr[K < kL ? K : kL] = v;
                    K += (i < (int)rn[q] && (reach || leave)) ? 1 : 0;
                }
            }
            // pad to a multiple of four with a disk that overlaps nothing
            // (entries stay below 8 CAP because K <= 8 CAP, a multiple of four)
            const int K4 = (K + 3) & ~3;
            const float2 far = make_float2(1.0e6f, 1.0e6f);
#pragma unroll
            for (int e = 0; e < 3; ++e)
                if (K + e < K4 && K + e < kL) nbr[K + e] = far;
            if (kO > 0 && K4 > kL) {
                int k2 = 0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (q == 4) continue;
#pragma unroll
                    for (int i = 0; i < CAP; ++i) {
                        bool reach;
                        const float2 v = frame_of(nv[q][i], q / 3, q % 3, g.wx, g.wy, reach);
                        const bool take = i < (int)rn[q] && (reach || leave);
                        if (take && k2 >= kL) ovf[k2 - kL] = v;
                        k2 += take ? 1 : 0;
                    }
                }
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if (K + e < K4 && K + e >= kL) ovf[K + e - kL] = far;
            }
            const int KL = K4 < kL ? K4 : kL;   // kL is a multiple of four
            // rng.shuffle(c.particles): Fisher-Yates over the stored list,
            // done on a packed permutation (nibble q = source slot of list
            // position q) and applied to the registers once.
            uint32_t P = 0x76543210u;
            const int nshuf = shuffle ? n - 1 : 0;
            for (int k = 0; k < nshuf; ++k) {
                if (k > 0 && (k & 3) == 0)
                    Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
                const int i = n - 1 - k;
                const int j = (int)bounded(word_of(Wsh, k & 3), (uint32_t)(i + 1));
                P = nib_swap(P, i, j);
            }
            if (nshuf > 0) {
                rperm(px, P);
                rperm(py, P);
                if (has_acc) {
                    rperm(ax, P);
                    rperm(ay, P);
                }
                if (has_tag) rperm(tg, P);
            }
            // 4. n_M trial moves on list[t mod n]: the registers are rotated
            // after every trial so that the particle moved is always entry 0.
            // The loop is uniform across the wave: the own-cell tests are
            // predicated arithmetic, and the neighbour groups run to the
            // wave's largest group count with each lane's own bound folded
            // into the test, so no lane-dependent branch or exec-mask update
            // sits in the loop.  (Which groups a lane tests, and in which
            // order, cannot change "some neighbour is closer than 1".)
            const int KLw = __ballot(KL >= 16) ? 16
                            : __ballot(KL >= 12) ? 12
                            : __ballot(KL >= 8) ? 8
                            : __ballot(KL >= 4) ? 4 : 0;
            // far entries up to the wave's group count and in the own-cell
            // slots past n, so that the trial loop needs no bounds at all
            for (int k = KL; k < KLw; ++k) nbr[k] = far;
#pragma unroll
            for (int q = 1; q < CAP; ++q) {
                px[q] = q < n ? px[q] : far.x;
                py[q] = q < n ? py[q] : far.y;
            }
            // the lane's row, read once into registers: the neighbours do not
            // move during the cell update, so the trials test registers only
            float2 nr[kL];
#pragma unroll
            for (int k = 0; k < kL; ++k) nr[k] = k < KLw ? nbr[k] : far;
            const int nm = leave_once ? n : n_moves;   // trial moves of this cell update
            for (int tr = 0; tr < nm; ++tr) {
                if (tr > 0 && (tr & 3) == 0) W = philox((uint32_t)c, s_lo, s_hi, (uint32_t)(tr >> 2), k0, k1);
                float dx, dy;
                if (disk)
                    disk_displacement(word_of(W, tr & 3), delta, dx, dy);
                else
                    displacement(word_of(W, tr & 3), delta, dx, dy);
                const float xm = px[0] + dx;
                const float ym = py[0] + dy;
                bool ok = (xm > lox) & (xm <= hix) & (ym > loy) & (ym <= hiy);
#pragma unroll
                for (int q = 1; q < CAP; ++q) {
                    const float ddx = xm - px[q];
                    const float ddy = ym - py[q];
                    const float r2 = pair_r2(ddx, ddy);
                    ok = ok & !(r2 < 1.0f);
                }
                // neighbours four at a time, up to the wave's group count
#pragma unroll
                for (int k = 0; k < kL; k += 4) {
                    if (k < KLw) {
                        const float m = min_r2(xm, ym, nr + k);
                        ok = ok & !(m < 1.0f);
                    }
                }
                if (kO > 0 && K4 > kL)
                    for (int k = kL; ok && k < K4; k += 4)
                        ok = !(min_r2(xm, ym, ovf + (k - kL)) < 1.0f);
                if (tr < 32) abits |= (ok ? 1u : 0u) << tr;
                px[0] = ok ? xm : px[0];
                py[0] = ok ? ym : py[0];
                if (has_acc) {
                    ax[0] = ok ? ax[0] + dx : ax[0];
                    ay[0] = ok ? ay[0] + dy : ay[0];
                }
                n_acc += ok ? 1u : 0u;
                rrot(px, n);   // the identity for n = 1
                rrot(py, n);
                if (has_acc) {
                    rrot(ax, n);
                    rrot(ay, n);
                }
                if (has_tag) rrot(tg, n);
            }
            n_trials = (unsigned)nm;
            // register entry q now holds list position (q + n_M) mod n
            const int r0 = nm % n;
#pragma unroll
            for (int q = 0; q < CAP; ++q) {
                if (q < n) {
                    int o = q + r0;
                    o = o >= n ? o - n : o;
                    pos[b0 + o] = make_float2(px[q], py[q]);
                    if (has_acc) acc[b0 + o] = make_float2(ax[q], ay[q]);
                    if (has_tag && n > 1) tag[b0 + o] = tg[q];
                }
            }
        }
    }
    if (alog && log_cell >= 0) alog[log_cell] = abits;
    // Counts are summed per wave (no barrier: a wave retires as soon as it is
    // done, not when the slowest wave of its workgroup is) and added to the
    // partial of the wave's 64-slot granule, which no other wave touches.
    const unsigned bt = wave_sum_u32(n_trials);
    const unsigned ba = wave_sum_u32(n_acc);
    if ((threadIdx.x & 63u) == 0 && tile < ntile && bt) {
        const long long gr = (slot0 + (long long)threadIdx.x) / kGranule;
        atomicAdd(&cnt[gr], (unsigned long long)bt);
        atomicAdd(&cnt[cnt_stride + gr], (unsigned long long)ba);
    }
}

// One wavefront per active cell (lanes_per_cell = 64): lane l < 9 CAP holds
// slot l % CAP of neighbourhood cell l / CAP (q = 3 row + col; the own cell
// is q = 4) in the cell's frame, and each trial is tested by every lane
// against its own entry, the verdicts combined by a wave ballot.  The moved
// disk's position is broadcast from the lane that holds it.  The chain is
// k_subsweep's -- the same draws, the same visit order, the same FP32 pair
// test and write-back order -- so the results are identical.  A wave does
// the work of one lane of k_subsweep, so this is the slow form; it is kept
// to measure that mapping against one lane per cell.  The cell-leaving
// pitfalls use the one-lane kernel.
template <int CAP, int PROP, bool ONE>
__global__ void __launch_bounds__(256)
k_subsweep_wave(Tables t, int par, float2 *__restrict__ pos, const uint32_t *__restrict__ count,
                float2 *__restrict__ acc, uint32_t *__restrict__ tag, uint32_t *__restrict__ alog,
                unsigned long long *__restrict__ cnt, int cnt_stride, int set, int ntile, int per)
{
    static_assert(9 * CAP <= 64, "one neighbourhood slot per lane");
    const int tile = xcd_tile(per);
    const int lane = (int)(threadIdx.x & 63u);
    const long long slot = (long long)tile * (blockDim.x / 64) + (long long)(threadIdx.x / 64);
    const int r = ONE ? 0 : chunk_replica(t, tile < ntile, slot / kActiveChunk);
    const Rep R = ONE ? t.rep0 : t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = t.ctls + r;
    const unsigned long long s = ctl->sweep_at[par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const int n_moves = R.n_moves;
    const bool disk = PROP == 2 ? R.disk != 0 : PROP == 1;
    const bool shuffle = PROP == 2 ? (R.ablate & kAblateParticleShuffle) == 0 : true;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);
    int Q = set;
    if (Q < 0) Q = (int)((ctl->draw_at[par].order >> (8 * (-1 - set))) & 0xFFu);
    const int qx = Q & 1, qy = Q >> 1;
    const int hx = g.mx >> 1, hy = g.my >> 1;
    const int gid = (int)(slot - R.ab);               // the wave's cell within the replica
    const uint32_t *const cn = count + R.cb;
    const size_t sb = (size_t)R.cb * CAP;
    unsigned n_trials = 0, n_acc = 0;
    uint32_t abits = 0;
    const bool valid = tile < ntile && gid < hx * hy;   // uniform across the wave
    if (valid) {
        const int iy = (int)((unsigned)gid / (unsigned)hx), ix = gid - iy * hx;
        const int cx = 2 * ix + qx, cy = 2 * iy + qy;
        const int c = cy * g.mx + cx;
        const int xl = cx == 0 ? g.mx - 1 : cx - 1;
        const int xr = cx == g.mx - 1 ? 0 : cx + 1;
        const int yd = cy == 0 ? g.my - 1 : cy - 1;
        const int yu = cy == g.my - 1 ? 0 : cy + 1;
        const bool holds = lane < 9 * CAP;
        const int q = holds ? lane / CAP : 4, i = holds ? lane % CAP : 0;
        const int row = q / 3 == 0 ? yd : (q / 3 == 1 ? cy : yu);
        const int col = q % 3 == 0 ? xl : (q % 3 == 1 ? cx : xr);
        const int cc = row * g.mx + col;
        const uint32_t rn = cn[cc];
        const float2 v = pos[sb + (size_t)cc * CAP + (size_t)i];
        const uint32_t n_raw = cn[c];
        uint4 Wsh = make_uint4(0, 0, 0, 0);
        if (shuffle) Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle, k0, k1);
        uint4 W = make_uint4(0, 0, 0, 0);
        if (n_moves > 0) W = philox((uint32_t)c, s_lo, s_hi, 0u, k0, k1);
        int n = (int)n_raw;
        if (__ballot(holds && rn > (uint32_t)g.cap) != 0ull) {
            if (lane == 0) atomicOr((unsigned int *)&ctl->errword, kErrCapacity);
            n = 0;
        }
        bool reach;
        const float2 f = frame_of(v, q / 3, q % 3, g.wx, g.wy, reach);
        const bool own = holds && q == 4 && i < n;        // a disk of the cell
        const bool nbr = holds && q != 4 && i < (int)rn;  // a disk of a neighbour cell
        if (n > 0) {
            const size_t b0 = sb + (size_t)c * CAP;
            const bool has_acc = acc != nullptr, has_tag = tag != nullptr;
            float px = f.x, py = f.y, ax = 0.0f, ay = 0.0f;
            uint32_t tg = 0u;
            if (has_acc && own) {
                const float2 a = acc[b0 + (size_t)i];
                ax = a.x;
                ay = a.y;
            }
            if (has_tag && own) tg = tag[b0 + (size_t)i];
            // rng.shuffle(c.particles) as a packed permutation: list
            // position p holds the disk of slot nibble p (the same on every lane)
            uint32_t P = 0x76543210u;
            const int nshuf = shuffle ? n - 1 : 0;
            for (int k = 0; k < nshuf; ++k) {
                if (k > 0 && (k & 3) == 0)
                    Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
                const int a = n - 1 - k;
                const int b = (int)bounded(word_of(Wsh, k & 3), (uint32_t)(a + 1));
                P = nib_swap(P, a, b);
            }
            for (int tr = 0; tr < n_moves; ++tr) {
                if (tr > 0 && (tr & 3) == 0) W = philox((uint32_t)c, s_lo, s_hi, (uint32_t)(tr >> 2), k0, k1);
                float dx, dy;
                if (disk)
                    disk_displacement(word_of(W, tr & 3), delta, dx, dy);
                else
                    displacement(word_of(W, tr & 3), delta, dx, dy);
                const int p = tr % n;                                   // list position moved
                const int L = 4 * CAP + (int)((P >> (4 * p)) & 0xFu);   // the lane holding it
                const float xm = __shfl(px, L, 64) + dx;
                const float ym = __shfl(py, L, 64) + dy;
                const bool in_cell = (xm > 0.0f) & (xm <= g.wx) & (ym > 0.0f) & (ym <= g.wy);
                const float ddx = xm - px, ddy = ym - py;
                const float r2 = pair_r2(ddx, ddy);
                const bool hit = (nbr || (own && lane != L)) && r2 < 1.0f;
                const bool ok = in_cell && __ballot(hit) == 0ull;
                if (tr < 32) abits |= (ok ? 1u : 0u) << tr;
                if (ok && lane == L) {
                    px = xm;
                    py = ym;
                    if (has_acc) {
                        ax = ax + dx;
                        ay = ay + dy;
                    }
                }
                n_acc += ok ? 1u : 0u;
            }
            n_trials = (unsigned)n_moves;
            // back to memory in list order: the disk of slot i goes to the
            // list position whose nibble is i
            if (own) {
                int o = 0;
#pragma unroll
                for (int k = 0; k < CAP; ++k) o = ((P >> (4 * k)) & 0xFu) == (uint32_t)i ? k : o;
                pos[b0 + (size_t)o] = make_float2(px, py);
                if (has_acc) acc[b0 + (size_t)o] = make_float2(ax, ay);
                if (has_tag && n > 1) tag[b0 + (size_t)o] = tg;
            }
        }
        if (alog && lane == 0) alog[R.cb + c] = abits;
    }
    if (lane == 0 && valid && n_trials) {
        const long long gr = slot / kGranule;
        atomicAdd(&cnt[gr], (unsigned long long)n_trials);
        atomicAdd(&cnt[cnt_stride + gr], (unsigned long long)n_acc);
    }
}

// The sub-sweep with LPC = 2 or 4 lanes per active cell: the same chain as
// k_subsweep, with the work that dominates a lane split across its group.
// Each lane loads the own cell and 8 / LPC of the neighbour cells (one
// corner and one edge cell per pair of them), filters and keeps those
// neighbours, and tests the trial positions against them; the group ANDs
// the verdicts (DPP), so every lane of the group sees the same accept
// decision and carries the same own-cell state.  Even lanes draw the cell's
// first trial block, odd lanes its first shuffle block, and the pair swaps
// them.  Every comparison is the one k_subsweep makes, so the results are
// identical; the gain is twice or four times the waves in flight, each with
// a shorter chain of dependent work, where a launch has too few cells to
// hide latency.
template <int CAP, int LPC, int PROP, bool ONE>
__global__ void __launch_bounds__(256)
k_subsweep_mc(Tables t, int par, float2 *__restrict__ pos, const uint32_t *__restrict__ count,
              float2 *__restrict__ acc, uint32_t *__restrict__ tag, uint32_t *__restrict__ alog,
              unsigned long long *__restrict__ cnt, int cnt_stride, float2 *__restrict__ ovf_all,
              int set, int ntile, int per)
{
    extern __shared__ float2 lds[];
    constexpr int NB = 8 / LPC;             // neighbour cells per lane
    constexpr int kE = NB * CAP;            // neighbour slots per lane
    constexpr int kL = kE < kNbrLds ? kE : kNbrLds;
    constexpr int kO = kE - kL;
    constexpr int kRow = kL + 1;
    const int tile = xcd_tile(per);
    const long long lane0 = (long long)tile * blockDim.x;
    const long long slot0 = lane0 / LPC;
    const int r = ONE ? 0 : chunk_replica(t, tile < ntile, slot0 / kActiveChunk);
    const Rep R = ONE ? t.rep0 : t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = t.ctls + r;
    const unsigned long long s = ctl->sweep_at[par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const int n_moves = R.n_moves;
    // proposal: fixed for the launch (PROP 0 square, 1 in-circle) or per
    // replica (PROP 2, which also carries the particle-shuffle ablation)
    const bool disk = PROP == 2 ? R.disk != 0 : PROP == 1;
    const bool shuffle = PROP == 2 ? (R.ablate & kAblateParticleShuffle) == 0 : true;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);

    int Q = set;
    if (Q < 0) Q = (int)((ctl->draw_at[par].order >> (8 * (-1 - set))) & 0xFFu);
    const int qx = Q & 1, qy = Q >> 1;
    const int hx = g.mx >> 1, hy = g.my >> 1;
    const int h = (int)(threadIdx.x % LPC);
    const int gid = (int)(slot0 - R.ab) + (int)(threadIdx.x / LPC);   // cell within the replica
    float2 *const nbr = lds + threadIdx.x * kRow;
    float2 *const ovf = ovf_all + (size_t)(lane0 + (long long)threadIdx.x) * kO;
    const uint32_t *const cn = count + R.cb;        // this replica's cell counts
    const size_t sb = (size_t)R.cb * CAP;           // and its first slot

    unsigned n_trials = 0, n_acc = 0;
    uint32_t abits = 0;
    long long log_cell = -1;   // global cell index of this lane's cell, if any
    if (tile < ntile && gid < hx * hy) {
        const int iy = (int)((unsigned)gid / (unsigned)hx), ix = gid - iy * hx;
        const int cx = 2 * ix + qx, cy = 2 * iy + qy;
        const int c = cy * g.mx + cx;
        log_cell = R.cb + c;
        const int xl = cx == 0 ? g.mx - 1 : cx - 1;
        const int xr = cx == g.mx - 1 ? 0 : cx + 1;
        const int yd = cy == 0 ? g.my - 1 : cy - 1;
        const int yu = cy == g.my - 1 ? 0 : cy + 1;
        // own cell and this lane's neighbour cells: q = 3 row + col over
        // {0, 1, 2, 3, 5, 6, 7, 8}, lane h taking entries h NB .. h NB + NB - 1;
        // counts and slots all in flight together
        const size_t b0 = sb + (size_t)c * CAP;   // own slots
        int n = (int)cn[c];
        float px[CAP], py[CAP];
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            const float2 v = pos[b0 + (size_t)i];
            px[i] = v.x;
            py[i] = v.y;
        }
        uint32_t rn[NB];
        int qa[NB];
        float2 nv[NB][CAP];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int e = h * NB + j;
            const int q = e < 4 ? e : e + 1;
            qa[j] = q;
            const int ra = q / 3, cb = q - 3 * (q / 3);
            const int row = ra == 0 ? yd : (ra == 1 ? cy : yu);
            const int col = cb == 0 ? xl : (cb == 1 ? cx : xr);
            const int cc = row * g.mx + col;
            rn[j] = cn[cc];
#pragma unroll
            for (int i = 0; i < CAP; ++i) nv[j][i] = pos[sb + (size_t)cc * CAP + (size_t)i];
        }
        // first trial block on even lanes, first shuffle block on odd lanes,
        // then swapped within the pair (computed while the loads fly)
        const uint4 mine = philox((uint32_t)c, s_lo, s_hi, (h & 1) ? kTagShuffle : 0u, k0, k1);
        const uint4 other = make_uint4(lane_xor1(mine.x), lane_xor1(mine.y), lane_xor1(mine.z),
                                       lane_xor1(mine.w));
        uint4 W = (h & 1) ? other : mine;
        uint4 Wsh = (h & 1) ? mine : other;
        bool bad = n > g.cap;
#pragma unroll
        for (int j = 0; j < NB; ++j) bad |= rn[j] > (uint32_t)g.cap;
        bad = group_any<LPC>(bad);
        if (bad) {
            if (h == 0) atomicOr((unsigned int *)&ctl->errword, kErrCapacity);
            n = 0;
        }
        if (n > 0) {
            const bool has_acc = acc != nullptr, has_tag = tag != nullptr;
            float ax[CAP], ay[CAP];
            uint32_t tg[CAP];
#pragma unroll
            for (int i = 0; i < CAP; ++i) {
                ax[i] = ay[i] = 0.0f;
                tg[i] = 0u;
            }
            if (has_acc) {
#pragma unroll
                for (int i = 0; i < CAP; ++i) {
                    const float2 a = acc[b0 + (size_t)i];
                    ax[i] = a.x;
                    ay[i] = a.y;
                }
            }
            if (has_tag) {
#pragma unroll
                for (int i = 0; i < CAP; ++i) tg[i] = tag[b0 + (size_t)i];
            }
            // this lane's neighbours in the cell's frame, reachable ones kept
            // (branch-free common path and rare overflow pass, as in k_subsweep)
            int K = 0;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int q = qa[j];
#pragma unroll
                for (int i = 0; i < CAP; ++i) {
                    bool reach;
                    const float2 v = frame_of(nv[j][i], q / 3, q - 3 * (q / 3), g.wx, g.wy, reach);
                    nbr[K < kL ? K : kL] = v;
                    K += (i < (int)rn[j] && reach) ? 1 : 0;
                }
            }
            const int K4 = (K + 3) & ~3;
            const float2 far = make_float2(1.0e6f, 1.0e6f);
#pragma unroll
            for (int e = 0; e < 3; ++e)
                if (K + e < K4 && K + e < kL) nbr[K + e] = far;
            if (kO > 0 && K4 > kL) {
                int k2 = 0;
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const int q = qa[j];
#pragma unroll
                    for (int i = 0; i < CAP; ++i) {
                        bool reach;
                        const float2 v =
                            frame_of(nv[j][i], q / 3, q - 3 * (q / 3), g.wx, g.wy, reach);
                        const bool take = i < (int)rn[j] && reach;
                        if (take && k2 >= kL) ovf[k2 - kL] = v;
                        k2 += take ? 1 : 0;
                    }
                }
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if (K + e < K4 && K + e >= kL) ovf[K + e - kL] = far;
            }
            const int KL = K4 < kL ? K4 : kL;
            uint32_t P = 0x76543210u;
            const int nshuf = shuffle ? n - 1 : 0;
            for (int k = 0; k < nshuf; ++k) {
                if (k > 0 && (k & 3) == 0)
                    Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
                const int i = n - 1 - k;
                const int j = (int)bounded(word_of(Wsh, k & 3), (uint32_t)(i + 1));
                P = nib_swap(P, i, j);
            }
            if (nshuf > 0) {
                rperm(px, P);
                rperm(py, P);
                if (has_acc) {
                    rperm(ax, P);
                    rperm(ay, P);
                }
                if (has_tag) rperm(tg, P);
            }
            for (int tr = 0; tr < n_moves; ++tr) {
                if (tr > 0 && (tr & 3) == 0) W = philox((uint32_t)c, s_lo, s_hi, (uint32_t)(tr >> 2), k0, k1);
                float dx, dy;
                if (disk)
                    disk_displacement(word_of(W, tr & 3), delta, dx, dy);
                else
                    displacement(word_of(W, tr & 3), delta, dx, dy);
                const float xm = px[0] + dx;
                const float ym = py[0] + dy;
                bool ok = xm > 0.0f && xm <= g.wx && ym > 0.0f && ym <= g.wy;
                if (ok) {
#pragma unroll
                    for (int q = 1; q < CAP; ++q) {
                        if (q < n) {
                            const float ddx = xm - px[q];
                            const float ddy = ym - py[q];
                            const float r2 = pair_r2(ddx, ddy);
                            ok = ok && !(r2 < 1.0f);
                        }
                    }
                }
                for (int k = 0; ok && k < KL; k += 4)
                    ok = !(min_r2(xm, ym, nbr + k) < 1.0f);
                if (kO > 0)
                    for (int k = kL; ok && k < K4; k += 4)
                        ok = !(min_r2(xm, ym, ovf + (k - kL)) < 1.0f);
                ok = group_all<LPC>(ok);
                if (ok) {
                    if (tr < 32) abits |= 1u << tr;
                    px[0] = xm;
                    py[0] = ym;
                    if (has_acc) {
                        ax[0] = ax[0] + dx;
                        ay[0] = ay[0] + dy;
                    }
                    ++n_acc;
                }
                if (n > 1) {
                    rrot(px, n);
                    rrot(py, n);
                    if (has_acc) {
                        rrot(ax, n);
                        rrot(ay, n);
                    }
                    if (has_tag) rrot(tg, n);
                }
            }
            n_trials = (unsigned)n_moves;
            // the group shares the writes: lane h stores list positions o
            // with o mod LPC == h
            const int r0 = n_moves % n;
#pragma unroll
            for (int q = 0; q < CAP; ++q) {
                if (q < n) {
                    int o = q + r0;
                    o = o >= n ? o - n : o;
                    if (o % LPC == h) {
                        pos[b0 + o] = make_float2(px[q], py[q]);
                        if (has_acc) acc[b0 + o] = make_float2(ax[q], ay[q]);
                        if (has_tag && n > 1) tag[b0 + o] = tg[q];
                    }
                }
            }
            if (h != 0) n_trials = n_acc = 0;   // counted once per cell
        }
    }
    if (alog && log_cell >= 0 && h == 0) alog[log_cell] = abits;
    const unsigned bt = wave_sum_u32(n_trials);   // per wave, no barrier
    const unsigned ba = wave_sum_u32(n_acc);
    if ((threadIdx.x & 63u) == 0 && tile < ntile && bt) {
        const long long gr = (slot0 + (long long)(threadIdx.x / LPC)) / kGranule;
        atomicAdd(&cnt[gr], (unsigned long long)bt);
        atomicAdd(&cnt[cnt_stride + gr], (unsigned long long)ba);
    }
}

// One workgroup per replica: add its granules' partials into its control
// block and clear them.
__global__ void __launch_bounds__(256) k_fold_counters(Tables t, unsigned long long *cnt, int stride)
{
    __shared__ unsigned long long sh[8];
    const Rep &R = t.reps[blockIdx.x];
    const long long g0 = R.ab / kGranule, g1 = (R.ab + R.apad) / kGranule;
    unsigned long long tr = 0, ac = 0;
    for (long long i = g0 + threadIdx.x; i < g1; i += blockDim.x) {
        tr += cnt[i];
        ac += cnt[stride + i];
        cnt[i] = 0ull;
        cnt[stride + i] = 0ull;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o, 64);
        ac += __shfl_xor(ac, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[wave] = tr;
        sh[4 + wave] = ac;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Ctl *ctl = t.ctls + blockIdx.x;
        ctl->trials += sh[0] + sh[1] + sh[2] + sh[3];
        ctl->accepts += sh[4] + sh[5] + sh[6] + sh[7];
    }
}

// ----------------------------------------------------------------- rebin
// Alg. 4 on the slot layout: new cell c holds the stayers of old c followed
// by the leavers of the old cell in direction f, both in old slot order.
// One thread per cell, tiles of 256 cells; a thread loads the counts and all
// CAP slots of both cells at once -- one memory round trip -- and writes its
// new list straight into the other buffer, so no scan is needed.  Each
// disk's decision is one rounded shifted coordinate tested against (0, w].
// The first workgroup of each replica writes the replica's sweep slot of
// the half it writes: the next sweep and its draws when the shift is the
// sweep's own, else a copy of the current slot.
struct RebinArgs {
    Tables t;
    const float2 *pos;
    const uint32_t *count;
    const float2 *acc;
    const uint32_t *tag;
    float2 *pos_out;
    uint32_t *count_out;
    float2 *acc_out;
    uint32_t *tag_out;
    int par;          // half read; the other is written
    int f;            // >= 0 explicit shift; < 0 each replica's own
    float d;
    int advance;
    int ntile;
    int per;
};

__device__ __forceinline__ float shifted(float v, bool minus, float d)
{
    return minus ? v - d : v + d;
}

template <int CAP, bool ONE>
__global__ void __launch_bounds__(kRebinTile) k_rebin(RebinArgs a)
{
    const int tile = xcd_tile(a.per);
    if (tile >= a.ntile) return;
    const long long cell0 = (long long)tile * kRebinTile;
    const int r = ONE ? 0 : tile_replica(a.t, true, tile);
    const Rep R = ONE ? a.t.rep0 : a.t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = a.t.ctls + r;
    int f = a.f;
    float d = a.d;
    if (f < 0) {
        f = ctl->draw_at[a.par].f;
        d = ctl->draw_at[a.par].d;
    }
    const bool along_x = f < 2;
    const bool minus = (f == 0 || f == 2);   // +x / +y: t = v - d
    const float w = along_x ? g.wx : g.wy;
    const float sw = minus ? w : -w;         // translation into the receiving cell

    const int cl = (int)(cell0 - R.cb) + (int)threadIdx.x;        // cell within the replica
    const bool valid = cl < g.C;
    unsigned stay = 0, leave = 0;   // bit i: own slot i stays / neighbour slot i leaves
    size_t ob = 0, nbb = 0;         // first slots of the two cells
    float2 own[CAP], nb[CAP];
    if (valid) {
        const int c = (int)cl;
        const int cy = c / g.mx, cx = c - cy * g.mx;
        int ncx = cx, ncy = cy;
        if (along_x) ncx = minus ? (cx == g.mx - 1 ? 0 : cx + 1) : (cx == 0 ? g.mx - 1 : cx - 1);
        else ncy = minus ? (cy == g.my - 1 ? 0 : cy + 1) : (cy == 0 ? g.my - 1 : cy - 1);
        const int nc = ncy * g.mx + ncx;
        ob = (size_t)(R.cb + c) * CAP;
        nbb = (size_t)(R.cb + nc) * CAP;
        int no = (int)a.count[R.cb + c];
        int nn = (int)a.count[R.cb + nc];
        // all CAP slots of both cells with the counts, one round trip
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            own[i] = a.pos[ob + (size_t)i];
            nb[i] = a.pos[nbb + (size_t)i];
        }
        if (no > g.cap || nn > g.cap) {
            atomicOr(&ctl->errword, kErrCapacity);
            no = no > g.cap ? g.cap : no;
            nn = nn > g.cap ? g.cap : nn;
        }
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            const float to = shifted(along_x ? own[i].x : own[i].y, minus, d);
            const float tn = shifted(along_x ? nb[i].x : nb[i].y, minus, d);
            if (i < no && to > 0.0f && to <= w) stay |= 1u << i;
            if (i < nn && !(tn > 0.0f && tn <= w)) leave |= 1u << i;
        }
    }
    const unsigned cnt = (unsigned)(__popc(stay) + __popc(leave));
    if (valid) {
        const bool has_acc = a.acc != nullptr, has_tag = a.tag != nullptr;
        if (cnt > (unsigned)g.cap) atomicOr(&ctl->errword, kErrCapacity);
        a.count_out[cell0 + threadIdx.x] = cnt > (unsigned)g.cap ? (unsigned)g.cap : cnt;
        // the new list of this cell, in its own CAP slots (never past them)
        size_t o = ob;
        const size_t oe = ob + (size_t)g.cap;
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            if ((stay & (1u << i)) && o < oe) {
                const float tt = shifted(along_x ? own[i].x : own[i].y, minus, d);
                a.pos_out[o] = along_x ? make_float2(tt, own[i].y) : make_float2(own[i].x, tt);
                if (has_acc) a.acc_out[o] = a.acc[ob + (size_t)i];
                if (has_tag) a.tag_out[o] = a.tag[ob + (size_t)i];
            }
            o += (stay >> i) & 1u;
        }
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            if ((leave & (1u << i)) && o < oe) {
                const float tt = shifted(along_x ? nb[i].x : nb[i].y, minus, d);
                const float t2 = tt + sw;
                a.pos_out[o] = along_x ? make_float2(t2, nb[i].y) : make_float2(nb[i].x, t2);
                if (has_acc) a.acc_out[o] = a.acc[nbb + (size_t)i];
                if (has_tag) a.tag_out[o] = a.tag[nbb + (size_t)i];
            }
            o += (leave >> i) & 1u;
        }
    } else if (cl < R.cpad) {
        a.count_out[cell0 + threadIdx.x] = 0u;   // padding cells stay empty
    }
    if (cell0 == R.cb && threadIdx.x == 0) {
        const unsigned long long s = ctl->sweep_at[a.par];
        if (a.advance) {
            store_draws(ctl, a.par ^ 1, s + 1ull, R);
        } else {
            ctl->sweep_at[a.par ^ 1] = s;
            ctl->draw_at[a.par ^ 1] = ctl->draw_at[a.par];
        }
    }
}

// The shift under the cell-leaving pitfalls (diagnostic): disks may sit up
// to (w - 1)/2 outside their cells on either axis.  One thread per new cell
// c: every disk of the 3x3 old cells gets its shifted coordinate (one FP32
// operation) and the other one; per axis a value <= 0 lands one cell down
// (coordinate + w), a value > w one cell up (coordinate - w).  The disks
// that land in c are listed: c's own first, then the eight neighbours' in
// row-major order of the offset, each in list order -- without excursions
// exactly k_rebin's order.
__device__ __forceinline__ int land(float t, float w, float &u)
{
    if (t <= 0.0f) {
        u = t + w;
        return -1;
    }
    if (t > w) {
        u = t - w;
        return 1;
    }
    u = t;
    return 0;
}

template <int CAP, bool ONE>
__global__ void __launch_bounds__(kRebinTile) k_rebin_general(RebinArgs a)
{
    const int tile = xcd_tile(a.per);
    if (tile >= a.ntile) return;
    const long long cell0 = (long long)tile * kRebinTile;
    const int r = ONE ? 0 : tile_replica(a.t, true, tile);
    const Rep R = ONE ? a.t.rep0 : a.t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = a.t.ctls + r;
    int f = a.f;
    float d = a.d;
    if (f < 0) {
        f = ctl->draw_at[a.par].f;
        d = ctl->draw_at[a.par].d;
    }
    const bool along_x = f < 2;
    const bool minus = (f == 0 || f == 2);   // +x / +y: t = v - d
    const int cl = (int)(cell0 - R.cb) + (int)threadIdx.x;   // cell within the replica
    if (cl < g.C) {
        const int cy = cl / g.mx, cx = cl - cy * g.mx;
        const bool has_acc = a.acc != nullptr, has_tag = a.tag != nullptr;
        const size_t ob = (size_t)(R.cb + cl) * CAP;
        int o = 0;
        bool over = false;
        for (int k = 0; k < 9; ++k) {
            const int q = k == 0 ? 4 : (k <= 4 ? k - 1 : k);
            const int ox = q % 3 - 1, oy = q / 3 - 1;
            const int sx = ox < 0 ? (cx == 0 ? g.mx - 1 : cx - 1) : (ox > 0 ? (cx == g.mx - 1 ? 0 : cx + 1) : cx);
            const int sy = oy < 0 ? (cy == 0 ? g.my - 1 : cy - 1) : (oy > 0 ? (cy == g.my - 1 ? 0 : cy + 1) : cy);
            const long long sc = R.cb + (long long)sy * g.mx + sx;
            int ns = (int)a.count[sc];
            if (ns > g.cap) {
                over = true;
                ns = g.cap;
            }
            for (int i = 0; i < ns; ++i) {
                const size_t si = (size_t)sc * CAP + (size_t)i;
                const float2 v = a.pos[si];
                const float tx = along_x ? shifted(v.x, minus, d) : v.x;
                const float ty = along_x ? v.y : shifted(v.y, minus, d);
                float ux, uy;
                const int mxo = land(tx, g.wx, ux);
                const int myo = land(ty, g.wy, uy);
                if (mxo != -ox || myo != -oy) continue;   // lands elsewhere
                if (o < g.cap) {
                    a.pos_out[ob + (size_t)o] = make_float2(ux, uy);
                    if (has_acc) a.acc_out[ob + (size_t)o] = a.acc[si];
                    if (has_tag) a.tag_out[ob + (size_t)o] = a.tag[si];
                } else {
                    over = true;
                }
                ++o;
            }
        }
        if (over) atomicOr(&ctl->errword, kErrCapacity);
        a.count_out[R.cb + cl] = (uint32_t)(o > g.cap ? g.cap : o);
    } else if (cl < R.cpad) {
        a.count_out[R.cb + cl] = 0u;   // padding cells stay empty
    }
    if (cell0 == R.cb && threadIdx.x == 0) {
        const unsigned long long s = ctl->sweep_at[a.par];
        if (a.advance) {
            store_draws(ctl, a.par ^ 1, s + 1ull, R);
        } else {
            ctl->sweep_at[a.par ^ 1] = s;
            ctl->draw_at[a.par ^ 1] = ctl->draw_at[a.par];
        }
    }
}

// ------------------------------------------------------- fused sweep
// A whole sweep (Alg. 1: the four sub-sweeps in the sweep's set order, then
// Alg. 4's shift and rebuild) in one launch, tile by tile.  A workgroup owns
// an interior of tx x ty cells of one replica (at most TILE x TILE) and
// loads it with a halo into LDS.  The rebuild of an interior cell c needs c
// and its neighbour in direction f after the four sub-sweeps: box B4, the
// interior extended by one cell towards f.  Sub-sweep p updates the cells
// of its set in B_p, B4 grown by 4 - p cells on every side, so that every
// update reads cells that already hold the state after sub-sweep p - 1; the
// region loaded is B1 grown by one cell (at most kFH = 5 around the
// interior).  A cell of the halo is updated by every tile that loads
// it, each time with the same neighbourhood and the same Philox stream
// (keyed by the cell and the sweep), so every copy ends identical to the one
// its owner computes: the result is the chain of the four separate launches,
// bit for bit, while the cells are read from and written to device memory
// once per sweep.  Only interior updates are counted (trials, accepts,
// accept bits).  Slots past a cell's count hold a far-away disk in LDS, so
// the overlap tests need no masks; the 3x3 neighbourhood is tested in full
// (no reach filter: with the data in LDS it costs what it saves).
// Accumulators and tags, when kept, live in LDS beside the positions and
// follow their disks; they take room, so the tile is smaller with them.
constexpr int kFH = 5;                   // halo: four sub-sweeps and the rebuild
constexpr int kFBlock = 512;             // lanes per workgroup
constexpr float kFar = 1.0e6f;

// Tile geometry.  LDS layout: the region split into its four parity planes
// (cell (rx, ry) in plane (rx & 1) + 2 (ry & 1) at (ry >> 1, rx >> 1)), one
// array per slot.  The active cells of a set are then consecutive in one
// plane, and so are each of their neighbours in the other planes: lanes
// read consecutive words, free of bank conflicts.
template <int TILE>
struct FTile {
    static constexpr int R = TILE + 2 * kFH;   // largest loaded region per side (even)
    static constexpr int PW = R / 2;           // plane width
    static constexpr int PS = PW * PW;         // plane size
    static constexpr int RC = 4 * PS;          // region cells
    __device__ static __forceinline__ int cell(int rx, int ry)
    {
        return ((rx & 1) + 2 * (ry & 1)) * PS + (ry >> 1) * PW + (rx >> 1);
    }
};

template <int CAP, int TILE, bool ACC, bool TAG>
constexpr size_t fused_lds_bytes()
{
    return (size_t)FTile<TILE>::RC *
           (CAP * sizeof(float2) * (ACC ? 2 : 1) + (TAG ? CAP * sizeof(uint32_t) : 0) + 1);
}

struct FusedArgs {
    Tables t;
    const float2 *pos;
    const uint32_t *count;
    const float2 *acc;
    const uint32_t *tag;
    float2 *pos_out;
    uint32_t *count_out;
    float2 *acc_out;
    uint32_t *tag_out;
    uint32_t *alog;
    unsigned long long *cnt;
    int cnt_stride;
    int par;
    int per;
};

// The LDS copy of a region: positions, optional accumulators and tags, counts.
template <int CAP, int TILE, bool ACC, bool TAG>
struct FRegion {
    float2 *sp;    // [CAP][RC]
    float2 *sa;    // [CAP][RC] (ACC)
    uint32_t *st;  // [CAP][RC] (TAG)
    uint8_t *sn;   // [RC]
    __device__ __forceinline__ FRegion(char *base)
    {
        constexpr int RC = FTile<TILE>::RC;
        sp = (float2 *)base;
        base += (size_t)RC * CAP * sizeof(float2);
        sa = (float2 *)base;
        if (ACC) base += (size_t)RC * CAP * sizeof(float2);
        st = (uint32_t *)base;
        if (TAG) base += (size_t)RC * CAP * sizeof(uint32_t);
        sn = (uint8_t *)base;
    }
};

// One cell update (Alg. 2) on the LDS copy of the region: cell (rx, ry) of
// the region, cell c of the replica.  The same decisions, in the same FP32
// operations, as k_subsweep.
template <int CAP, int TILE, bool ACC, bool TAG>
__device__ __forceinline__ void fused_cell_update(const FRegion<CAP, TILE, ACC, TAG> &L, int rx,
                                                  int ry, uint32_t c, float wx, float wy,
                                                  uint32_t s_lo, uint32_t s_hi, uint32_t k0,
                                                  uint32_t k1, float delta, int n_moves,
                                                  bool disk, bool shuffle, unsigned &n_acc,
                                                  uint32_t &abits)
{
    using G = FTile<TILE>;
    const int r = G::cell(rx, ry);
    const int n = (int)L.sn[r];
    if (n == 0) return;
    uint4 Wsh = make_uint4(0, 0, 0, 0);
    if (shuffle && n > 1) Wsh = philox(c, s_lo, s_hi, kTagShuffle, k0, k1);
    uint4 W = make_uint4(0, 0, 0, 0);
    if (n_moves > 0) W = philox(c, s_lo, s_hi, 0u, k0, k1);
    float px[CAP], py[CAP], ax[CAP], ay[CAP];
    uint32_t tg[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        const float2 v = L.sp[i * G::RC + r];
        px[i] = v.x;
        py[i] = v.y;
        ax[i] = ay[i] = 0.0f;
        tg[i] = 0u;
        if (ACC) {
            const float2 u = L.sa[i * G::RC + r];
            ax[i] = u.x;
            ay[i] = u.y;
        }
        if (TAG) tg[i] = L.st[i * G::RC + r];
    }
    // the eight neighbours' slots in this cell's frame (exactly -w, 0, +w)
    float nx[8 * CAP], ny[8 * CAP];
#pragma unroll
    for (int q = 0, e = 0; q < 9; ++q) {
        if (q == 4) continue;
        const int ra = q / 3, cb = q % 3;
        const int rq = G::cell(rx + cb - 1, ry + ra - 1);
#pragma unroll
        for (int i = 0; i < CAP; ++i, ++e) {
            const float2 v = L.sp[i * G::RC + rq];
            float ox = v.x, oy = v.y;
            if (cb == 0) ox = ox - wx;
            if (cb == 2) ox = ox + wx;
            if (ra == 0) oy = oy - wy;
            if (ra == 2) oy = oy + wy;
            nx[e] = ox;
            ny[e] = oy;
        }
    }
    // rng.shuffle(c.particles) as a packed permutation of the first n
    // entries (entries >= n, far disks, stay in place)
    uint32_t P = 0x76543210u;
    const int nshuf = shuffle ? n - 1 : 0;
    for (int k = 0; k < nshuf; ++k) {
        if (k > 0 && (k & 3) == 0)
            Wsh = philox(c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
        const int i = n - 1 - k;
        const int j = (int)bounded(word_of(Wsh, k & 3), (uint32_t)(i + 1));
        P = nib_swap(P, i, j);
    }
    if (nshuf > 0) {
        rperm(px, P);
        rperm(py, P);
        if (ACC) {
            rperm(ax, P);
            rperm(ay, P);
        }
        if (TAG) rperm(tg, P);
    }
    for (int tr = 0; tr < n_moves; ++tr) {
        if (tr > 0 && (tr & 3) == 0) W = philox(c, s_lo, s_hi, (uint32_t)(tr >> 2), k0, k1);
        float dx, dy;
        if (disk)
            disk_displacement(word_of(W, tr & 3), delta, dx, dy);
        else
            displacement(word_of(W, tr & 3), delta, dx, dy);
        const float xm = px[0] + dx;
        const float ym = py[0] + dy;
        bool ok = (xm > 0.0f) & (xm <= wx) & (ym > 0.0f) & (ym <= wy);
#pragma unroll
        for (int q = 1; q < CAP; ++q) {
            const float ddx = xm - px[q];
            const float ddy = ym - py[q];
            const float r2 = pair_r2(ddx, ddy);
            ok = ok & !(r2 < 1.0f);
        }
#pragma unroll
        for (int e = 0; e < 8 * CAP; e += 4) {
            const float d0x = xm - nx[e], d0y = ym - ny[e];
            const float d1x = xm - nx[e + 1], d1y = ym - ny[e + 1];
            const float d2x = xm - nx[e + 2], d2y = ym - ny[e + 2];
            const float d3x = xm - nx[e + 3], d3y = ym - ny[e + 3];
            const float m = fminf(fminf(pair_r2(d0x, d0y), pair_r2(d1x, d1y)),
                                  fminf(pair_r2(d2x, d2y), pair_r2(d3x, d3y)));
            ok = ok & !(m < 1.0f);
        }
        if (tr < 32) abits |= (ok ? 1u : 0u) << tr;
        px[0] = ok ? xm : px[0];
        py[0] = ok ? ym : py[0];
        if (ACC) {
            ax[0] = ok ? ax[0] + dx : ax[0];
            ay[0] = ok ? ay[0] + dy : ay[0];
        }
        n_acc += ok ? 1u : 0u;
        rrot(px, n);
        rrot(py, n);
        if (ACC) {
            rrot(ax, n);
            rrot(ay, n);
        }
        if (TAG) rrot(tg, n);
    }
    // register entry q holds list position (q + n_M) mod n: back to LDS in
    // list order (slots >= n keep their far entries)
    const int r0 = n_moves % n;
#pragma unroll
    for (int o = 0; o < CAP; ++o) {
        if (o < n) {
            int q = o - r0;
            q = q < 0 ? q + n : q;
            L.sp[o * G::RC + r] = make_float2(rsel(px, q), rsel(py, q));
            if (ACC) L.sa[o * G::RC + r] = make_float2(rsel(ax, q), rsel(ay, q));
            if (TAG) L.st[o * G::RC + r] = rsel(tg, q);
        }
    }
}

__device__ __forceinline__ int wrap_once(int v, int m) { return v < 0 ? v + m : (v >= m ? v - m : v); }

template <int CAP, int PROP, bool ONE, int TILE, bool ACC, bool TAG>
__global__ void __launch_bounds__(kFBlock, 2) k_sweep_fused(FusedArgs a)
{
    using G = FTile<TILE>;
    extern __shared__ char lds_fb[];
    const FRegion<CAP, TILE, ACC, TAG> L(lds_fb);
    const int tile = xcd_tile(a.per);
    if (tile >= a.t.ftiles) return;
    const int r = ONE ? 0 : (int)a.t.trep[tile];
    const Rep R = ONE ? a.t.rep0 : a.t.reps[r];
    const Geom g = R.g;
    Ctl *ctl = a.t.ctls + r;
    const int lt = tile - (int)R.tb;            // tile within the replica
    const int tyi = lt / R.tiles_x, txi = lt - tyi * R.tiles_x;
    const int x0 = txi * a.t.ftx, y0 = tyi * a.t.fty;
    const int wI = min(a.t.ftx, g.mx - x0), hI = min(a.t.fty, g.my - y0);
    const unsigned long long s = ctl->sweep_at[a.par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const uint32_t order = ctl->draw_at[a.par].order;
    const int f = ctl->draw_at[a.par].f;
    const float d = ctl->draw_at[a.par].d;
    const int n_moves = R.n_moves;
    const bool disk = PROP == 2 ? R.disk != 0 : PROP == 1;
    const bool shuffle = PROP == 2 ? (R.ablate & kAblateParticleShuffle) == 0 : true;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);
    const uint32_t *cn = a.count + R.cb;
    const size_t sb = (size_t)R.cb * CAP;   // the replica's first slot
    // direction of the rebuild's neighbour and the box B4 it needs (region
    // column rx is column x0 - kFH + rx)
    const bool along_x = f < 2;
    const bool minus = (f == 0 || f == 2);   // +x / +y: t = v - d
    const int ddx = along_x ? (minus ? 1 : -1) : 0;
    const int ddy = along_x ? 0 : (minus ? 1 : -1);
    const int b4x0 = kFH + min(ddx, 0), b4x1 = kFH + wI + max(ddx, 0);
    const int b4y0 = kFH + min(ddy, 0), b4y1 = kFH + hI + max(ddy, 0);

    // load the region: cell (rx, ry) is cell ((x0 - kFH + rx) mod mx,
    // (y0 - kFH + ry) mod my) (grids narrower than the halo wrap twice);
    // slots past the count hold a far disk
    bool bad = false;
    const int lx0 = b4x0 - 4, ly0 = b4y0 - 4;
    const int LX = b4x1 + 4 - lx0, LY = b4y1 + 4 - ly0;
    for (int i = threadIdx.x; i < LX * LY; i += kFBlock) {
        const int iy = i / LX;
        const int rx = lx0 + (i - iy * LX), ry = ly0 + iy;
        const int gx = wrap_once(wrap_once(x0 - kFH + rx, g.mx), g.mx);
        const int gy = wrap_once(wrap_once(y0 - kFH + ry, g.my), g.my);
        const int c = gy * g.mx + gx;
        uint32_t n = cn[c];
        float2 v[CAP], u[CAP];
        uint32_t tv[CAP];
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            v[k] = a.pos[sb + (size_t)c * CAP + k];
            if (ACC) u[k] = a.acc[sb + (size_t)c * CAP + k];
            if (TAG) tv[k] = a.tag[sb + (size_t)c * CAP + k];
        }
        if (n > (uint32_t)g.cap) {
            bad = true;
            n = 0;
        }
        const int rr = G::cell(rx, ry);
        L.sn[rr] = (uint8_t)n;
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            L.sp[k * G::RC + rr] = k < (int)n ? v[k] : make_float2(kFar, kFar);
            if (ACC) L.sa[k * G::RC + rr] = u[k];
            if (TAG) L.st[k * G::RC + rr] = tv[k];
        }
    }
    if (bad) atomicOr((unsigned int *)&ctl->errword, kErrCapacity);
    __syncthreads();

    // four sub-sweeps, each on its set's cells of a box one cell smaller
    unsigned n_trials = 0, n_acc = 0;
#pragma unroll 1
    for (int p = 1; p <= 4; ++p) {
        const int Q = (int)((order >> (8 * (p - 1))) & 0xFFu);
        const int qx = Q & 1, qy = Q >> 1;
        const int bx0 = b4x0 - (4 - p), bx1 = b4x1 + (4 - p);
        const int by0 = b4y0 - (4 - p), by1 = b4y1 + (4 - p);
        // region column rx is column x0 - kFH + rx (x0 even): parity of rx + 1
        const int fx = bx0 + (((bx0 + 1) ^ qx) & 1), fy = by0 + (((by0 + 1) ^ qy) & 1);
        const int nxa = (bx1 - fx + 1) >> 1, nya = (by1 - fy + 1) >> 1;
        for (int i = threadIdx.x; i < nxa * nya; i += kFBlock) {
            const int iy = i / nxa, ix = i - iy * nxa;
            const int rx = fx + 2 * ix, ry = fy + 2 * iy;
            const int gx = wrap_once(wrap_once(x0 - kFH + rx, g.mx), g.mx);
            const int gy = wrap_once(wrap_once(y0 - kFH + ry, g.my), g.my);
            const uint32_t c = (uint32_t)(gy * g.mx + gx);
            const bool inner = rx >= kFH && rx < kFH + wI && ry >= kFH && ry < kFH + hI;
            unsigned acc_here = 0;
            uint32_t bits = 0;
            const int nbefore = (int)L.sn[G::cell(rx, ry)];
            fused_cell_update<CAP, TILE, ACC, TAG>(L, rx, ry, c, g.wx, g.wy, s_lo, s_hi, k0, k1,
                                                   delta, n_moves, disk, shuffle, acc_here, bits);
            if (inner) {
                n_acc += acc_here;
                n_trials += nbefore > 0 ? (unsigned)n_moves : 0u;
                if (a.alog) a.alog[R.cb + c] = bits;
            }
        }
        __syncthreads();
    }

    // the shift and rebuild (Alg. 4) of the interior: new cell c holds the
    // stayers of c, then the leavers of its neighbour in direction f
    const float w = along_x ? g.wx : g.wy;
    const float swd = minus ? w : -w;
    bool over = false;
    for (int i = threadIdx.x; i < wI * hI; i += kFBlock) {
        const int iy = i / wI, ix = i - iy * wI;
        const int rx = kFH + ix, ry = kFH + iy;
        const int ro = G::cell(rx, ry), rn = G::cell(rx + ddx, ry + ddy);
        const int no = (int)L.sn[ro], nn = (int)L.sn[rn];
        // candidates in list order (own slots, then the neighbour's), each
        // kept by its one rounded shifted coordinate; kept candidate i goes
        // to output slot popcount(keep below i)
        float2 cand[2 * CAP], cacc[2 * CAP];
        uint32_t ctag[2 * CAP];
        uint32_t keep = 0u;
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            const float2 v = L.sp[k * G::RC + ro];
            const float tt = shifted(along_x ? v.x : v.y, minus, d);
            cand[k] = along_x ? make_float2(tt, v.y) : make_float2(v.x, tt);
            if (ACC) cacc[k] = L.sa[k * G::RC + ro];
            if (TAG) ctag[k] = L.st[k * G::RC + ro];
            keep |= (k < no && tt > 0.0f && tt <= w) ? 1u << k : 0u;
        }
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            const float2 v = L.sp[k * G::RC + rn];
            const float tt = shifted(along_x ? v.x : v.y, minus, d);
            const float t2 = tt + swd;
            cand[CAP + k] = along_x ? make_float2(t2, v.y) : make_float2(v.x, t2);
            if (ACC) cacc[CAP + k] = L.sa[k * G::RC + rn];
            if (TAG) ctag[CAP + k] = L.st[k * G::RC + rn];
            keep |= (k < nn && !(tt > 0.0f && tt <= w)) ? 1u << (CAP + k) : 0u;
        }
        float2 out[CAP], oacc[CAP];
        uint32_t otag[CAP];
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            out[k] = make_float2(kFar, kFar);
            oacc[k] = make_float2(0.0f, 0.0f);
            otag[k] = 0u;
        }
#pragma unroll
        for (int i = 0; i < 2 * CAP; ++i) {
            const bool kk = (keep >> i) & 1u;
            const int idx = __popc(keep & ((1u << i) - 1u));
#pragma unroll
            for (int j = 0; j < CAP; ++j) {
                const bool here = kk && idx == j;
                out[j] = here ? cand[i] : out[j];
                if (ACC) oacc[j] = here ? cacc[i] : oacc[j];
                if (TAG) otag[j] = here ? ctag[i] : otag[j];
            }
        }
        int o = __popc(keep);
        if (o > g.cap) {
            over = true;
            o = g.cap;
        }
        const int c = (y0 + iy) * g.mx + (x0 + ix);
        a.count_out[R.cb + c] = (uint32_t)o;
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
            a.pos_out[sb + (size_t)c * CAP + k] = out[k];
            if (ACC) a.acc_out[sb + (size_t)c * CAP + k] = oacc[k];
            if (TAG) a.tag_out[sb + (size_t)c * CAP + k] = otag[k];
        }
    }
    if (over) atomicOr((unsigned int *)&ctl->errword, kErrCapacity);
    // padding cells of the replica (beyond C) keep count 0 in the half written
    if (lt == 0)
        for (long long i = g.C + threadIdx.x; i < R.cpad; i += kFBlock) a.count_out[R.cb + i] = 0u;
    // counts per wave into a granule of the replica (folded on demand)
    const unsigned bt = wave_sum_u32(n_trials);
    const unsigned ba = wave_sum_u32(n_acc);
    if ((threadIdx.x & 63u) == 0 && bt) {
        const long long ng = R.apad / kGranule;
        const long long gr = R.ab / kGranule + ((long long)lt * (kFBlock / 64) + threadIdx.x / 64) % ng;
        atomicAdd(&a.cnt[gr], (unsigned long long)bt);
        atomicAdd(&a.cnt[a.cnt_stride + gr], (unsigned long long)ba);
    }
    if (lt == 0 && threadIdx.x == 0) store_draws(ctl, a.par ^ 1, s + 1ull, R);
}

// ------------------------------------------------------ pair histogram
// Ordered pairs (k, j != k) within reach, r^2 in k's frame as in the trial
// moves, binned on E_b = (float)((1 + b 1e-4)^2) (Sec. 4).  Tiles of 256
// cells, so each workgroup belongs to one replica and adds into its
// histogram.
__global__ void __launch_bounds__(kRebinTile)
k_pair_hist(Tables t, const float2 *__restrict__ pos, const uint32_t *__restrict__ count,
            int ntile, int per)
{
    __shared__ float E[kHistBins + 1];
    __shared__ unsigned H[kHistBins];
    for (int i = threadIdx.x; i <= kHistBins; i += blockDim.x) {
        const double rr = 1.0 + (double)i * 1e-4;
        E[i] = (float)(rr * rr);
        if (i < kHistBins) H[i] = 0;
    }
    __syncthreads();
    const int tile = xcd_tile(per);
    const long long cell0 = (long long)tile * kRebinTile;
    const int r = tile_replica(t, tile < ntile, tile);
    const Rep R = rep_of(t, r);
    const Geom g = R.g;
    const double rmax = 1.0 + kHistBins * 1e-4;
    const int Rx = (double)g.wx >= rmax ? 1 : 2;
    const int Ry = (double)g.wy >= rmax ? 1 : 2;
    const uint32_t *const cn = count + R.cb;
    const float2 *const pr = pos + (size_t)R.cb * t.cap;   // slots: t.cap per cell
    const long long cl = cell0 + (long long)threadIdx.x - R.cb;
    if (tile < ntile && cl < g.C) {
        const int c = (int)cl;
        const int cy = c / g.mx, cx = c - cy * g.mx;
        const float e0 = E[0], eN = E[kHistBins];
        const uint32_t nk = min(cn[c], (uint32_t)g.cap);   // counts trusted only up to capacity
        for (uint32_t k = 0; k < nk; ++k) {
            const float2 pk = pr[(size_t)c * t.cap + k];
            for (int oy = -Ry; oy <= Ry; ++oy) {
                const int ncy = (cy + oy + 2 * g.my) % g.my;
                const float ty = (float)oy * g.wy;
                for (int ox = -Rx; ox <= Rx; ++ox) {
                    const int ncx = (cx + ox + 2 * g.mx) % g.mx;
                    const float tx = (float)ox * g.wx;
                    const int nc = ncy * g.mx + ncx;
                    for (uint32_t j = 0, je = min(cn[nc], (uint32_t)g.cap); j < je; ++j) {
                        if (nc == c && j == k) continue;
                        const float2 v = pr[(size_t)nc * t.cap + j];
                        const float qx = v.x + tx;
                        const float qy = v.y + ty;
                        const float ddx = pk.x - qx;
                        const float ddy = pk.y - qy;
                        const float r2 = ddx * ddx + ddy * ddy;
                        if (r2 < e0 || r2 >= eN) continue;
                        int lo = 0, hi = kHistBins;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (r2 >= E[mid]) lo = mid;
                            else hi = mid;
                        }
                        atomicAdd(&H[lo], 1u);
                    }
                }
            }
        }
    }
    __syncthreads();
    if (tile < ntile) {
        Ctl *ctl = t.ctls + r;
        for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
            if (H[i]) atomicAdd(&ctl->hist[i], (unsigned long long)H[i]);
        if (cell0 == R.cb && threadIdx.x == 0) atomicAdd(&ctl->hist_samples, 1ull);
    }
}

__global__ void k_hist_reset(Tables t)
{
    Ctl *ctl = t.ctls + blockIdx.x;
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0ull;
    if (threadIdx.x == 0) ctl->hist_samples = 0ull;
}

// ------------------------------------------------------ contact fit (FP64)
// g(R_i) from Eq. gR at the Eq. R points, unweighted least squares of a
// degree-5 polynomial in (R - 1)/0.02 by Householder QR, P* from Eq. P.
__global__ void __launch_bounds__(256) k_pressure_fit(Tables t, int replica)
{
    constexpr int NB = kHistBins, NC = 6;
    __shared__ double A[NB][NC];
    __shared__ double y[NB];
    __shared__ double v[NB];
    const Geom g = t.reps[replica].g;
    Ctl *ctl = t.ctls + replica;
    const unsigned long long S = ctl->hist_samples;
    const double box_x = (double)g.mx * (double)g.wx;
    const double box_y = (double)g.my * (double)g.wy;
    const double rho = (double)g.N / (box_x * box_y);
    const double dr = 1e-4, cfit = 0.02, pi = 3.14159265358979323846;
    for (int i = threadIdx.x; i < NB; i += blockDim.x) {
        const double r0 = 1.0 + (double)i * dr;
        const double r1 = 1.0 + (double)(i + 1) * dr;
        const double Ri = (2.0 / 3.0) * (r1 * r1 * r1 - r0 * r0 * r0) / (r1 * r1 - r0 * r0);
        const double n = (double)ctl->hist[i] / (double)(S ? S : 1ull);
        y[i] = n / ((double)g.N * rho * 2.0 * pi * Ri * dr);
        const double x = (Ri - 1.0) / cfit;
        double xp = 1.0;
        for (int k = 0; k < NC; ++k) {
            A[i][k] = xp;
            xp *= x;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (S == 0) {
        ctl->fit[3] = -1.0;
        return;
    }
    for (int k = 0; k < NC; ++k) {
        double norm2 = 0.0;
        for (int i = k; i < NB; ++i) norm2 += A[i][k] * A[i][k];
        const double norm = sqrt(norm2);
        const double alpha = A[k][k] > 0.0 ? -norm : norm;
        double vn2 = 0.0;
        for (int i = k; i < NB; ++i) {
            v[i] = A[i][k] - (i == k ? alpha : 0.0);
            vn2 += v[i] * v[i];
        }
        if (vn2 == 0.0) continue;
        for (int j = k; j < NC; ++j) {
            double dot = 0.0;
            for (int i = k; i < NB; ++i) dot += v[i] * A[i][j];
            const double sc = 2.0 * dot / vn2;
            for (int i = k; i < NB; ++i) A[i][j] -= sc * v[i];
        }
        double dot = 0.0;
        for (int i = k; i < NB; ++i) dot += v[i] * y[i];
        const double sc = 2.0 * dot / vn2;
        for (int i = k; i < NB; ++i) y[i] -= sc * v[i];
    }
    double coef[NC];
    for (int k = NC - 1; k >= 0; --k) {
        double acc = y[k];
        for (int j = k + 1; j < NC; ++j) acc -= A[k][j] * coef[j];
        coef[k] = acc / A[k][k];
    }
    ctl->fit[0] = rho * (1.0 + 0.5 * pi * rho * coef[0]);
    ctl->fit[1] = coef[0];
    ctl->fit[2] = rho;
    ctl->fit[3] = 1.0;
}

// ------------------------------------------------------ overlap count
// A pair overlaps when r^2 < 1 - 2^-20 in either disk's frame.  The trial
// moves test r^2 < 1 in the mover's frame; seen from the partner's frame the
// same pair can round to 1 - a few ulp of r^2, and every rebin re-expresses
// a coordinate with one rounding (at most 2^-24 absolute for values below
// 2) while neither disk moves, so the invariant allows 2^-20.
constexpr float kOverlapR2 = 1.0f - 0x1p-20f;

__global__ void __launch_bounds__(kRebinTile)
k_count_overlaps(Tables t, const float2 *__restrict__ pos, const uint32_t *__restrict__ count,
                 int ntile, int per)
{
    __shared__ unsigned red[16];
    const int tile = xcd_tile(per);
    const long long cell0 = (long long)tile * kRebinTile;
    const int r = tile_replica(t, tile < ntile, tile);
    const Rep R = rep_of(t, r);
    const Geom g = R.g;
    const uint32_t *const cn = count + R.cb;
    const float2 *const pr = pos + (size_t)R.cb * t.cap;   // slots: t.cap per cell
    const long long cl = cell0 + (long long)threadIdx.x - R.cb;
    unsigned bad = 0;
    if (tile < ntile && cl < g.C) {
        const int c = (int)cl;
        const int cy = c / g.mx, cx = c - cy * g.mx;
        const uint32_t nk = min(cn[c], (uint32_t)g.cap);   // counts trusted only up to capacity
        for (uint32_t k = 0; k < nk; ++k) {
            const float2 pk = pr[(size_t)c * t.cap + k];
            for (int oy = -1; oy <= 1; ++oy) {
                const int ncy = (cy + oy + g.my) % g.my;
                const float ty = oy < 0 ? -g.wy : (oy > 0 ? g.wy : 0.0f);
                for (int ox = -1; ox <= 1; ++ox) {
                    const int ncx = (cx + ox + g.mx) % g.mx;
                    const float tx = ox < 0 ? -g.wx : (ox > 0 ? g.wx : 0.0f);
                    const int nc = ncy * g.mx + ncx;
                    for (uint32_t j = 0, je = min(cn[nc], (uint32_t)g.cap); j < je; ++j) {
                        if (nc == c && j == k) continue;
                        const float2 v = pr[(size_t)nc * t.cap + j];
                        const float ddx = pk.x - (v.x + tx);
                        const float ddy = pk.y - (v.y + ty);
                        bad += (ddx * ddx + ddy * ddy < kOverlapR2) ? 1u : 0u;
                    }
                }
            }
        }
    }
    const unsigned tot = block_sum_u32(bad, red);
    if (threadIdx.x == 0 && tile < ntile && tot)
        atomicAdd((unsigned long long *)&t.ctls[r].overlaps, (unsigned long long)tot);
}

__global__ void k_overlaps_reset(Tables t) { t.ctls[blockIdx.x].overlaps = 0; }

// ------------------------------------------------------------- MSD
// Deterministic FP64 reduction of |acc|^2 over a replica's disks, in cell
// and slot order (the order of the compact lists): one workgroup per
// replica, each thread a fixed stride of slots, a fixed tree at the end.
constexpr int kMsdThreads = 256;
constexpr int kMsdBlocks = kMsdBlocksMax;

// One replica over kMsdBlocks workgroups: workgroup b sums a fixed range of
// cells, the final kernel adds the partials in order.
__global__ void __launch_bounds__(kMsdThreads)
k_msd_partial(Tables t, int r, const float2 *__restrict__ acc, const uint32_t *__restrict__ count,
              double *__restrict__ part)
{
    __shared__ double sh[kMsdThreads];
    const Rep R = rep_of(t, r);
    const long long S = t.cap;
    const long long chunk = ((long long)R.g.C + gridDim.x - 1) / gridDim.x;
    const long long c0 = (long long)blockIdx.x * chunk;
    const long long c1 = c0 + chunk < R.g.C ? c0 + chunk : (long long)R.g.C;
    const float2 *a = acc + (size_t)R.cb * S;
    const uint32_t *cn = count + R.cb;
    double s = 0.0;
    for (long long i = c0 * S + threadIdx.x; i < c1 * S; i += kMsdThreads) {
        const long long c = i / S;
        if (i - c * S < (long long)cn[c]) {
            const float2 v = a[i];
            s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kMsdThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kMsdThreads)
k_msd_final(const double *__restrict__ part, int nb, long long N, Ctl *ctl)
{
    __shared__ double sh[kMsdThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->msd = N > 0 ? sh[0] / (double)N : 0.0;
}

// Every replica, one workgroup each.
__global__ void __launch_bounds__(kMsdThreads)
k_msd_all(Tables t, const float2 *__restrict__ acc, const uint32_t *__restrict__ count)
{
    __shared__ double sh[kMsdThreads];
    const Rep R = rep_of(t, blockIdx.x);
    const long long S = t.cap;
    const long long slots = (long long)R.g.C * S;
    const float2 *a = acc + (size_t)R.cb * S;
    const uint32_t *cn = count + R.cb;
    double s = 0.0;
    for (long long i = threadIdx.x; i < slots; i += kMsdThreads) {
        const long long c = i / S;
        if (i - c * S < (long long)cn[c]) {
            const float2 v = a[i];
            s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kMsdThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) t.ctls[blockIdx.x].msd = R.g.N > 0 ? sh[0] / (double)R.g.N : 0.0;
}

// ------------------------------------------------------------- tuner
// Per replica: delta <- delta * clamp(a / 0.3, 0.5, 2), clamped to
// [1e-3, min(w)/2], with a the acceptance of the window since the last
// update (FP64).
__global__ void k_tune(Tables t, int apply)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= t.R) return;
    Ctl *ctl = t.ctls + r;
    const Geom g = t.reps[r].g;
    const unsigned long long tr = ctl->trials - ctl->win_trials;
    const unsigned long long a = ctl->accepts - ctl->win_accepts;
    if (apply && tr > 0) {
        const double ratio = (double)a / (double)tr;
        double q = ratio / 0.3;
        if (q < 0.5) q = 0.5;
        if (q > 2.0) q = 2.0;
        double nd = (double)ctl->delta * q;
        const double hi = 0.5 * (double)(g.wx < g.wy ? g.wx : g.wy);
        if (nd < 1e-3) nd = 1e-3;
        if (nd > hi) nd = hi;
        ctl->delta = (float)nd;
    }
    ctl->win_trials = ctl->trials;
    ctl->win_accepts = ctl->accepts;
}

// ------------------------------------------------------------- utility
__global__ void k_fill_u32(uint32_t *p, uint32_t value, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// One workgroup per replica (first + blockIdx.x).
__global__ void k_ctl_reset(Tables t, int first, unsigned long long sweep)
{
    const int r = first + (int)blockIdx.x;
    Ctl *ctl = t.ctls + r;
    const Rep &R = t.reps[r];
    if (threadIdx.x == 0) {
        ctl->trials = ctl->accepts = 0ull;
        ctl->win_trials = ctl->win_accepts = 0ull;
        ctl->key0 = R.key0;
        ctl->key1 = R.key1;
        ctl->delta = R.delta0;
        ctl->errword = 0u;
        ctl->hist_samples = 0ull;
        ctl->overlaps = 0;
        ctl->msd = 0.0;
        for (int i = 0; i < 4; ++i) ctl->fit[i] = 0.0;
        store_draws(ctl, 0, sweep, R);
        store_draws(ctl, 1, sweep, R);
    }
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0ull;
}

__global__ void k_ctl_set_key0(Tables t, unsigned int key0)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= t.R) return;
    Ctl *ctl = t.ctls + r;
    ctl->key0 = key0;
    store_draws(ctl, 0, ctl->sweep_at[0], t.reps[r]);
    store_draws(ctl, 1, ctl->sweep_at[1], t.reps[r]);
}

__global__ void k_ctl_set_delta(Tables t, int first, int count, float delta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) t.ctls[first + i].delta = delta;
}

inline int tiles_for(long long items, int block) { return (int)((items + block - 1) / block); }
inline int per_xcd(int ntile) { return (ntile + 7) / 8; }

}  // namespace

// ================================================================ launches
// Workgroup size of the sub-sweep: the requested one, reduced if the LDS
// neighbour rows would exceed 64 KB (they do not for rows of 17 float2);
// always one of 64, 128, 192, 256, so it divides the active chunk.
int subsweep_block(int cap, int block, int lanes)
{
    const int e = 8 / lanes * cap;
    const int row = (e < kNbrLds ? e : kNbrLds) + 1;
    const int fit = (65536 / (row * (int)sizeof(float2))) / 64 * 64;
    return block < fit ? block : fit;
}

hipError_t launch_subsweep(const Tables &t, int par, float2 *pos, const uint32_t *count,
                           float2 *acc, uint32_t *tag, uint32_t *alog, const Work &w, int set,
                           int block, int lanes, hipStream_t st)
{
    if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 64) return hipErrorInvalidValue;
    if (t.leave) lanes = 1;   // the cell-leaving pitfalls run on the one-lane kernel only
    block = subsweep_block(t.cap, block, lanes);
    if (block < 64 || block > 256 || block % 64 || (kActiveChunk * lanes) % block)
        return hipErrorInvalidValue;
    const int ntile = tiles_for(t.active * lanes, block);
    const int per = per_xcd(ntile);
    const dim3 grid(8 * per), blk(block);
    const int e = 8 / lanes * t.cap;
    const int row = (e < kNbrLds ? e : kNbrLds) + 1;
    const size_t lds = lanes == 64 ? 0 : (size_t)row * block * sizeof(float2);
#define MPMC_SUB1(CAP, PROP, ONE)                                                              \
    do {                                                                                       \
        if (lanes == 64)                                                                       \
            hipLaunchKernelGGL((k_subsweep_wave<CAP, PROP, ONE>), grid, blk, 0, st, t, par, pos, \
                               count, acc, tag, alog, w.cnt, w.cnt_stride, set, ntile, per);   \
        else if (lanes == 1)                                                                   \
            hipLaunchKernelGGL((k_subsweep<CAP, PROP, ONE>), grid, blk, lds, st, t, par, pos,    \
                               count, acc, tag, alog, w.cnt, w.cnt_stride, w.ovf, set, ntile,  \
                               per);                                                           \
        else if (lanes == 2)                                                                   \
            hipLaunchKernelGGL((k_subsweep_mc<CAP, 2, PROP, ONE>), grid, blk, lds, st, t, par,   \
                               pos, count, acc, tag, alog, w.cnt, w.cnt_stride, w.ovf, set,    \
                               ntile, per);                                                    \
        else                                                                                   \
            hipLaunchKernelGGL((k_subsweep_mc<CAP, 4, PROP, ONE>), grid, blk, lds, st, t, par,   \
                               pos, count, acc, tag, alog, w.cnt, w.cnt_stride, w.ovf, set,    \
                               ntile, per);                                                    \
    } while (0)
#define MPMC_SUB(CAP, PROP)                                                                    \
    do {                                                                                       \
        if (t.R == 1) MPMC_SUB1(CAP, PROP, true);                                              \
        else MPMC_SUB1(CAP, PROP, false);                                                      \
    } while (0)
#define MPMC_SUB_P(CAP)                                                                        \
    do {                                                                                       \
        if (t.prop == 0) MPMC_SUB(CAP, 0);                                                     \
        else if (t.prop == 1) MPMC_SUB(CAP, 1);                                                \
        else MPMC_SUB(CAP, 2);                                                                 \
    } while (0)
    if (t.prop < 0 || t.prop > 2) return hipErrorInvalidValue;
    switch (t.cap) {
    case 4: MPMC_SUB_P(4); break;
    case 5: MPMC_SUB_P(5); break;
    case 6: MPMC_SUB_P(6); break;
    case 7: MPMC_SUB_P(7); break;
    default: return hipErrorInvalidValue;
    }
#undef MPMC_SUB_P
#undef MPMC_SUB
#undef MPMC_SUB1
    return hipGetLastError();
}

hipError_t launch_fold_counters(const Tables &t, const Work &w, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold_counters, dim3(t.R), dim3(256), 0, st, t, w.cnt, w.cnt_stride);
    return hipGetLastError();
}

int fused_tile(bool acc, bool tag) { return tag ? 20 : (acc ? 24 : 38); }

bool sweep_fused_supported(const Tables &t) { return t.cap == 4 && t.ftiles > 0 && !t.leave; }

hipError_t launch_sweep_fused(const Tables &t, int par, const float2 *pos, const uint32_t *count,
                              const float2 *acc, const uint32_t *tag, float2 *pos_out,
                              uint32_t *count_out, float2 *acc_out, uint32_t *tag_out,
                              uint32_t *alog, const Work &w, hipStream_t st)
{
    if (!sweep_fused_supported(t)) return hipErrorInvalidValue;
    const bool A = acc != nullptr, T = tag != nullptr;
    if (t.ftile != fused_tile(A, T)) return hipErrorInvalidValue;
    FusedArgs a;
    a.t = t;
    a.pos = pos;
    a.count = count;
    a.acc = acc;
    a.tag = tag;
    a.pos_out = pos_out;
    a.count_out = count_out;
    a.acc_out = acc_out;
    a.tag_out = tag_out;
    a.alog = alog;
    a.cnt = w.cnt;
    a.cnt_stride = w.cnt_stride;
    a.par = par;
    a.per = per_xcd((int)t.ftiles);
    const dim3 grid(8 * a.per), blk(kFBlock);
#define MPMC_FUSED(PROP, ONE, TL, AC, TG)                                                      \
    hipLaunchKernelGGL((k_sweep_fused<4, PROP, ONE, TL, AC, TG>), grid, blk,                    \
                       (fused_lds_bytes<4, TL, AC, TG>()), st, a)
#define MPMC_FUSED_F(PROP, ONE)                                                                \
    do {                                                                                       \
        if (T && A) MPMC_FUSED(PROP, ONE, 20, true, true);                                     \
        else if (T) MPMC_FUSED(PROP, ONE, 20, false, true);                                    \
        else if (A) MPMC_FUSED(PROP, ONE, 24, true, false);                                    \
        else MPMC_FUSED(PROP, ONE, 38, false, false);                                          \
    } while (0)
#define MPMC_FUSED_P(ONE)                                                                      \
    do {                                                                                       \
        if (t.prop == 0) MPMC_FUSED_F(0, ONE);                                                 \
        else if (t.prop == 1) MPMC_FUSED_F(1, ONE);                                            \
        else MPMC_FUSED_F(2, ONE);                                                             \
    } while (0)
    if (t.R == 1) MPMC_FUSED_P(true);
    else MPMC_FUSED_P(false);
#undef MPMC_FUSED_P
#undef MPMC_FUSED_F
#undef MPMC_FUSED
    return hipGetLastError();
}

hipError_t launch_rebin(const Tables &t, int par, const float2 *pos, const uint32_t *count,
                        const float2 *acc, const uint32_t *tag, float2 *pos_out,
                        uint32_t *count_out, float2 *acc_out, uint32_t *tag_out,
                        const Work &w, int f, float d, int advance, hipStream_t st)
{
    (void)w;
    RebinArgs a;
    a.t = t;
    a.par = par;
    a.pos = pos; a.count = count; a.acc = acc; a.tag = tag;
    a.pos_out = pos_out; a.count_out = count_out; a.acc_out = acc_out; a.tag_out = tag_out;
    a.f = f; a.d = d;
    a.advance = (f < 0 && advance) ? 1 : 0;
    a.ntile = tiles_for(t.cells, kRebinTile);
    a.per = per_xcd(a.ntile);
    const dim3 grid(8 * a.per), blk(kRebinTile);
#define MPMC_REBIN(CAP)                                                                        \
    do {                                                                                       \
        if (t.leave) {                                                                         \
            if (t.R == 1) hipLaunchKernelGGL((k_rebin_general<CAP, true>), grid, blk, 0, st, a); \
            else hipLaunchKernelGGL((k_rebin_general<CAP, false>), grid, blk, 0, st, a);       \
        } else if (t.R == 1) {                                                                 \
            hipLaunchKernelGGL((k_rebin<CAP, true>), grid, blk, 0, st, a);                     \
        } else {                                                                               \
            hipLaunchKernelGGL((k_rebin<CAP, false>), grid, blk, 0, st, a);                    \
        }                                                                                      \
    } while (0)
    switch (t.cap) {
    case 4: MPMC_REBIN(4); break;
    case 5: MPMC_REBIN(5); break;
    case 6: MPMC_REBIN(6); break;
    case 7: MPMC_REBIN(7); break;
    default: return hipErrorInvalidValue;
    }
#undef MPMC_REBIN
    return hipGetLastError();
}

hipError_t launch_pair_histogram(const Tables &t, const float2 *pos, const uint32_t *count,
                                 int reset, hipStream_t st)
{
    if (reset) hipLaunchKernelGGL(k_hist_reset, dim3(t.R), dim3(256), 0, st, t);
    const int ntile = tiles_for(t.cells, kRebinTile);
    const int per = per_xcd(ntile);
    hipLaunchKernelGGL(k_pair_hist, dim3(8 * per), dim3(kRebinTile), 0, st, t, pos, count, ntile, per);
    return hipGetLastError();
}

hipError_t launch_pressure_fit(const Tables &t, int replica, hipStream_t st)
{
    hipLaunchKernelGGL(k_pressure_fit, dim3(1), dim3(256), 0, st, t, replica);
    return hipGetLastError();
}

hipError_t launch_count_overlaps(const Tables &t, const float2 *pos, const uint32_t *count,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_overlaps_reset, dim3(t.R), dim3(1), 0, st, t);
    const int ntile = tiles_for(t.cells, kRebinTile);
    const int per = per_xcd(ntile);
    hipLaunchKernelGGL(k_count_overlaps, dim3(8 * per), dim3(kRebinTile), 0, st, t, pos, count,
                       ntile, per);
    return hipGetLastError();
}

hipError_t launch_msd(const Tables &t, int replica, long long N, const float2 *acc,
                      const uint32_t *count, const Work &w, hipStream_t st)
{
    hipLaunchKernelGGL(k_msd_partial, dim3(kMsdBlocks), dim3(kMsdThreads), 0, st, t, replica, acc,
                       count, w.f64);
    hipLaunchKernelGGL(k_msd_final, dim3(1), dim3(kMsdThreads), 0, st, w.f64, kMsdBlocks, N,
                       t.ctls + replica);
    return hipGetLastError();
}

hipError_t launch_msd_all(const Tables &t, const float2 *acc, const uint32_t *count, hipStream_t st)
{
    hipLaunchKernelGGL(k_msd_all, dim3(t.R), dim3(kMsdThreads), 0, st, t, acc, count);
    return hipGetLastError();
}

hipError_t launch_tune(const Tables &t, int apply, hipStream_t st)
{
    hipLaunchKernelGGL(k_tune, dim3((t.R + 63) / 64), dim3(64), 0, st, t, apply);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_ctl_reset(const Tables &t, int replica, unsigned long long sweep, hipStream_t st)
{
    const int first = replica < 0 ? 0 : replica;
    const int count = replica < 0 ? t.R : 1;
    hipLaunchKernelGGL(k_ctl_reset, dim3(count), dim3(256), 0, st, t, first, sweep);
    return hipGetLastError();
}

hipError_t launch_ctl_set_key0(const Tables &t, unsigned int key0, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctl_set_key0, dim3((t.R + 63) / 64), dim3(64), 0, st, t, key0);
    return hipGetLastError();
}

hipError_t launch_ctl_set_delta(const Tables &t, int replica, float delta, hipStream_t st)
{
    const int first = replica < 0 ? 0 : replica;
    const int count = replica < 0 ? t.R : 1;
    hipLaunchKernelGGL(k_ctl_set_delta, dim3((count + 63) / 64), dim3(64), 0, st, t, first, count,
                       delta);
    return hipGetLastError();
}

}  // namespace mpmc
