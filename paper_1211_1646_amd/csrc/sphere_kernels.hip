// HIP kernels of the hard-sphere chain (the method in d = 3) for gfx950.
//
// Method: Anderson et al., arXiv:1211.1646, stated for d dimensions (Sec. 2):
// Alg. 1 (sweep) over 8 checkerboard sets, Alg. 2 (cell update) against the
// 27-cell neighbourhood, Alg. 4 (cell shift) along one of 6 directions, and
// the contact-value pressure of Sec. 4 in its 3D form.
//
// Data layout in device memory:
//   count[C]    uint32 spheres per cell, c = (cz m_y + cy) m_x + cx;
//   pos[8 C]    float4 (x, y, z, 0) cell-local coordinates in (0, w], slots
//               [0, count) used: slots 0..1 of cell c in its 32-byte primary
//               line at 2 c, slots 2..7 in an overflow region at 2 C + 6 c
//               (slot_of).  The fourth word of slot 0 holds the bits of the
//               cell's count, also when the cell is empty, so that one
//               32-byte line gives a cell's count and first two spheres;
//   tag[8 C]    uint32 identity of each sphere (optional), same slots;
//   acc[8 C]    float4 displacement accumulated by accepted moves (optional),
//               same slots.
// A sub-sweep writes only the active cells' own slots and reads their 26
// inactive neighbours, so it updates in place; the rebin writes the other
// ping-pong half.
//
// Every floating-point expression rounds once per operation (the library is
// built with -ffp-contract=off; the pragma below repeats it).
#include "mpmc_device.h"
#include "sphere_internal.h"

#pragma clang fp contract(off)

namespace mpmc {
namespace sph {
namespace {

constexpr uint32_t kTagShuffle = 0x40000000u;
constexpr uint32_t kTagSweep = 0x80000000u;
constexpr uint32_t kCellGlobal = 0xFFFFFFFFu;

// One 16-bit half h of a trial word: the midpoint (2h + 1 - 65536) / 65536
// of one of 65536 equal parts of (-1, 1).
__device__ __forceinline__ float half_unit(uint32_t h)
{
    return (float)(2 * (int)h + 1 - 65536) * 0x1p-16f;
}

// Trial displacement from words a, b: x and y from the halves of a, z from
// the high half of b, each times delta.
__device__ __forceinline__ void displacement3(uint32_t a, uint32_t b, float delta, float &dx,
                                              float &dy, float &dz)
{
    dx = half_unit(a >> 16) * delta;
    dy = half_unit(a & 0xFFFFu) * delta;
    dz = half_unit(b >> 16) * delta;
}

struct Draws3 {
    uint32_t order;   // nibble q = set processed in slot q
    int f;
    float d;
};

// Draws of sweep s (Alg. 1 in d = 3): Fisher-Yates order of the 8 sets from
// words u0..u6 of two global blocks, f = floor(6 u7 / 2^32), d = u (w_f / 2)
// from the low 24 bits of word 0 of a third block.  The order is kept as
// eight nibbles of one register, so nothing is indexed at run time.
__device__ __forceinline__ Draws3 sweep_draws3(unsigned long long s, uint32_t k0, uint32_t k1,
                                               const Geom3 &g)
{
    const uint32_t lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
    const uint4 A = philox(kCellGlobal, lo, hi, kTagSweep, k0, k1);
    const uint4 B = philox(kCellGlobal, lo, hi, kTagSweep + 1u, k0, k1);
    const uint4 G = philox(kCellGlobal, lo, hi, kTagSweep + 2u, k0, k1);
    const uint32_t u[8] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w};
    uint32_t ord = 0x76543210u;
#pragma unroll
    for (int i = 7; i >= 1; --i) ord = nib_swap(ord, i, (int)bounded(u[7 - i], (uint32_t)(i + 1)));
    Draws3 D;
    D.order = ord;
    D.f = (int)bounded(u[7], 6u);
    const float wf = D.f < 2 ? g.w[0] : (D.f < 4 ? g.w[1] : g.w[2]);
    const float ud = (float)(G.x & 0xFFFFFFu) * 0x1p-24f;
    D.d = ud * (0.5f * wf);
    return D;
}

__device__ __forceinline__ void store_draws3(Ctl3 *ctl, int p, unsigned long long s,
                                             const Geom3 &g)
{
    const Draws3 D = sweep_draws3(s, ctl->key0, ctl->key1, g);
    ctl->sweep_at[p] = s;
    ctl->draw_at[p].order = D.order;
    ctl->draw_at[p].f = D.f;
    ctl->draw_at[p].d = D.d;
}

__device__ __forceinline__ int wrap_dn(int c, int m) { return c == 0 ? m - 1 : c - 1; }
__device__ __forceinline__ int wrap_up(int c, int m) { return c == m - 1 ? 0 : c + 1; }

// ------------------------------------------------------------ sub-sweep
// A group of LPC = 1, 2 or 4 lanes per active cell of set Q (Alg. 2 in
// d = 3).  Every lane of a group holds the cell's own spheres and draws the
// same random numbers; lane h takes neighbour cells h NB .. h NB + NB - 1
// of the 26 (NB = ceil(26 / LPC)), and a trial is accepted when every lane
// of the group finds no overlap (a DPP vote):
//   1. in one round trip: the own count and 8 slots, and the count and
//      first slot (first two with four lanes per cell) of each of the lane's
//      neighbour cells; the cell's first Philox blocks are computed while
//      they are in flight;
//   2. the further slots are loaded slot by slot (slot i of all the lane's
//      cells in one batch, only while some lane of the wave has a cell with
//      more than i spheres); every neighbour is translated into the cell's
//      frame by exactly -w, 0 or +w, and those that can reach a trial
//      position -- squared distance below 1.0001 to the box that holds
//      every trial position of this update (the cell's spheres' bounding
//      box grown by the most they can move, cut to the cell), a superset of
//      every sphere a trial can overlap -- are compacted into this lane's
//      column of an LDS table;
//   3. the column is read back into registers and the n_M trials run from
//      registers only.  A lane with more reachable neighbours than its
//      column holds also tests every neighbour straight from memory (rare).
// Dropping unreachable spheres cannot change a decision: a trial outside
// the cell is rejected before any overlap test, and one inside it lies in
// the box, at squared distance >= 1 from every dropped sphere, also after
// FP32 rounding.
constexpr float kReach2 = 1.0001f;
constexpr float kFar = 1.0e6f;
// Buffer descriptor word 3 of the gfx9 family (raw, range-checked 32-bit
// dwords), and an offset past the end of any slot array: the geometry check
// keeps C * 8 * 16 bytes below 2^31.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kPastEnd = 0x7FFFFFF0;

// Smallest r^2 from (xm, ym, zm) to entries k .. k+3; some r^2 < 1 iff the
// smallest is (all values finite).
__device__ __forceinline__ float min_r2_4(float xm, float ym, float zm, const float *ex,
                                          const float *ey, const float *ez)
{
    float m = 3.0e38f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float dx = xm - ex[e];
        const float dy = ym - ey[e];
        const float dz = zm - ez[e];
        m = fminf(m, pair_r2(dx, dy, dz));
    }
    return m;
}

// Neighbour offset o in {-1, 0, +1} applied to a coordinate (adding 0 is
// skipped: v + 0 == v for v > 0).
__device__ __forceinline__ float frame(float v, int o, float w)
{
    return o < 0 ? v - w : (o > 0 ? v + w : v);
}
__device__ __forceinline__ float gap(float v, int o, float w)
{
    return o < 0 ? -v : (o > 0 ? v - w : 0.0f);
}

// The rare path: does (xm, ym, zm) overlap any sphere of the 26 neighbour
// cells?  Reads counts and slots from memory (they do not change during the
// sub-sweep: no active cell is another's neighbour).
__device__ bool overlap_from_memory(const Geom3 &g, const float4 *__restrict__ pos,
                                    const uint32_t *__restrict__ count, int cx, int cy, int cz,
                                    float xm, float ym, float zm)
{
    bool hit = false;
    for (int q = 0; q < 27 && !hit; ++q) {
        if (q == 13) continue;
        const int ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
        const int nx = ox < 0 ? wrap_dn(cx, g.m[0]) : (ox > 0 ? wrap_up(cx, g.m[0]) : cx);
        const int ny = oy < 0 ? wrap_dn(cy, g.m[1]) : (oy > 0 ? wrap_up(cy, g.m[1]) : cy);
        const int nz = oz < 0 ? wrap_dn(cz, g.m[2]) : (oz > 0 ? wrap_up(cz, g.m[2]) : cz);
        const int nc = (nz * g.m[1] + ny) * g.m[0] + nx;
        const uint32_t cn = min(count[nc], (uint32_t)kCap);
        for (uint32_t j = 0; j < cn; ++j) {
            const float4 v = pos[slot_of(g.C, nc, (int)j)];
            const float dx = xm - frame(v.x, ox, g.w[0]);
            const float dy = ym - frame(v.y, oy, g.w[1]);
            const float dz = zm - frame(v.z, oz, g.w[2]);
            hit |= pair_r2(dx, dy, dz) < 1.0f;
        }
    }
    return hit;
}

// The cell (cx, cy, cz) shifted by o in {-1, 0, +1} per axis, as a cell index.
__device__ __forceinline__ int cell_at(const Geom3 &g, const int X[3], const int Y[3],
                                       const int Z[3], int ox, int oy, int oz)
{
    const int x = ox < 0 ? X[0] : (ox > 0 ? X[2] : X[1]);
    const int y = oy < 0 ? Y[0] : (oy > 0 ? Y[2] : Y[1]);
    const int z = oz < 0 ? Z[0] : (oz > 0 ? Z[2] : Z[1]);
    return (z * g.m[1] + y) * g.m[0] + x;
}

template <int LPC, bool ACC>
__global__ void __launch_bounds__(kSubBlock)
k_subsweep3(Geom3 g, Ctl3 *__restrict__ ctl, int par, float4 *__restrict__ pos,
            const uint32_t *__restrict__ count, uint32_t *__restrict__ tag,
            float4 *__restrict__ acc, unsigned long long *__restrict__ cnt, int set, int ntile,
            int per)
{
    constexpr int NB = (26 + LPC - 1) / LPC;                  // neighbour cells per lane
    constexpr int kL = LPC == 1 ? kNbrList : (LPC == 2 ? 24 : 16);   // LDS list per lane
    // slots loaded with the counts: never past the primary line
    constexpr int kU = (LPC == 4 ? 2 : 1) < kPrim ? (LPC == 4 ? 2 : 1) : kPrim;
    // entry k of lane l at [k][l] (the 64 lanes of a wave read 64 consecutive
    // words); row kL is a pad row that takes the writes of dropped entries,
    // so that no write needs a branch
    __shared__ float lx[kL + 1][kSubBlock];
    __shared__ float ly[kL + 1][kSubBlock];
    __shared__ float lz[kL + 1][kSubBlock];
    const int tile = xcd_tile(per);
    const int lane = threadIdx.x;
    const int h = lane % LPC;                                 // rank in the lane group
    const int a = (tile * kSubBlock + lane) / LPC;            // active cell of the group
    unsigned n_trials = 0, n_acc = 0;
    const bool live = tile < ntile && a < g.active;
    const unsigned long long s = ctl->sweep_at[par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);
    int Q = set;
    if (Q < 0) Q = (int)((ctl->draw_at[par].order >> (4 * (-1 - set))) & 0xFu);
    const int hx = g.m[0] >> 1, hy = g.m[1] >> 1;
    const int aa = live ? a : 0;   // a lane past the end reads cell 0's block and drops it
    const int ix = aa % hx, iy = (aa / hx) % hy, iz = aa / (hx * hy);
    const int cx = 2 * ix + (Q & 1), cy = 2 * iy + ((Q >> 1) & 1), cz = 2 * iz + (Q >> 2);
    const int X[3] = {wrap_dn(cx, g.m[0]), cx, wrap_up(cx, g.m[0])};
    const int Y[3] = {wrap_dn(cy, g.m[1]), cy, wrap_up(cy, g.m[1])};
    const int Z[3] = {wrap_dn(cz, g.m[2]), cz, wrap_up(cz, g.m[2])};
    const int c = (cz * g.m[1] + cy) * g.m[0] + cx;
    const size_t b0 = (size_t)c * kPrim;   // the own primary line

    // 1. in one round trip: the own count and slots, and for each of this
    // lane's neighbour cells (entries h NB .. h NB + NB - 1 of the 26, in
    // the order q = 9 (oz+1) + 3 (oy+1) + (ox+1) without the centre) its
    // count and its first kU slots.  Every address is inside the grid, so
    // the loads are issued unconditionally and masked afterwards.
    const uint32_t n_raw = live ? count[c] : 0u;
    float px[kCap], py[kCap], pz[kCap];
    uint32_t tg[kCap];
#pragma unroll
    for (int q = 0; q < kCap; ++q) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (q < kPrim) v = pos[b0 + (size_t)q];   // the primary line, unconditionally
        px[q] = v.x;
        py[q] = v.y;
        pz[q] = v.z;
        tg[q] = 0u;
    }
    const bool has_tag = tag != nullptr;
    if (has_tag) {
#pragma unroll
        for (int q = 0; q < kPrim; ++q) tg[q] = tag[b0 + (size_t)q];
    }
    // accumulators are a compile-time variant, so that the plain chain
    // carries no registers for them
    constexpr bool has_acc = ACC;
    float ax[kCap], ay[kCap], az[kCap];
#pragma unroll
    for (int q = 0; q < kCap; ++q) ax[q] = ay[q] = az[q] = 0.0f;
    if (has_acc) {
#pragma unroll
        for (int q = 0; q < kPrim; ++q) {
            const float4 v = acc[b0 + (size_t)q];
            ax[q] = v.x;
            ay[q] = v.y;
            az[q] = v.z;
        }
    }
    int cq[NB], oq[NB];       // neighbour cell and its offset code q
    uint32_t nn[NB];
    float4 v0[NB][kU];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int e = h * NB + j;
        const bool valid = live && e < 26;
        const int q = e < 13 ? e : e + 1;
        oq[j] = q;
        const int cell = cell_at(g, X, Y, Z, q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1);
        cq[j] = cell;
        const uint32_t cnt_j = count[cell];
        nn[j] = valid ? cnt_j : 0u;
#pragma unroll
        for (int u = 0; u < kU; ++u) v0[j][u] = pos[slot_of(g.C, cell, u)];
    }
    uint4 Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle, k0, k1);
    uint4 W = make_uint4(0, 0, 0, 0);
    if (g.n_moves > 0) W = philox((uint32_t)c, s_lo, s_hi, 0u, k0, k1);
    bool bad = n_raw > (uint32_t)kCap;
    uint32_t nmax = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        bad |= nn[j] > (uint32_t)kCap;
        nmax = max(nmax, nn[j]);
    }
    if (bad) atomicOr(&ctl->errword, kErrCapacity);
    // a cell above capacity anywhere in the group's block: skip the update
    const bool skip = group_any<LPC>(bad);
    const int n = skip ? 0 : (int)n_raw;
    if (n == 0) nmax = 0;
    nmax = min(nmax, (uint32_t)kCap);

    // own overflow slots, only where some lane of the wave has more than kPrim
    // spheres (out-of-range offsets read nothing for the others)
    const __amdgpu_buffer_rsrc_t slots = __builtin_amdgcn_make_buffer_rsrc(
        (void *)pos, (short)0, (int)((unsigned)g.C * (unsigned)(kCap * sizeof(float4))), kBufferWord3);
    if (__ballot(n > kPrim) != 0ull) {
#pragma unroll
        for (int q = kPrim; q < kCap; ++q) {
            const int off = n > q ? (int)slot_of(g.C, c, q) * (int)sizeof(float4) : kPastEnd;
            const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(slots, off, 0, 0));
            px[q] = v.x;
            py[q] = v.y;
            pz[q] = v.z;
            if (has_tag && n > q) tg[q] = tag[slot_of(g.C, c, q)];
            if (has_acc && n > q) {
                const float4 u = acc[slot_of(g.C, c, q)];
                ax[q] = u.x;
                ay[q] = u.y;
                az[q] = u.z;
            }
        }
    }

    // The box that holds every trial position of this cell update: a sphere
    // of the cell moves at most k = ceil(n_M / n) times, each time by at most
    // delta per axis (plus a rounding of at most 1e-7 here), and a trial
    // outside the cell is rejected before any overlap test.  The margin
    // 1e-5 covers the rounding of the box itself.
    float blo[3] = {0.0f, 0.0f, 0.0f}, bhi[3] = {g.w[0], g.w[1], g.w[2]};
    if (n > 0) {
        float mn[3] = {px[0], py[0], pz[0]}, mx[3] = {px[0], py[0], pz[0]};
#pragma unroll
        for (int q = 1; q < kCap; ++q) {
            const bool in = q < n;
            mn[0] = in ? fminf(mn[0], px[q]) : mn[0];
            mx[0] = in ? fmaxf(mx[0], px[q]) : mx[0];
            mn[1] = in ? fminf(mn[1], py[q]) : mn[1];
            mx[1] = in ? fmaxf(mx[1], py[q]) : mx[1];
            mn[2] = in ? fminf(mn[2], pz[q]) : mn[2];
            mx[2] = in ? fmaxf(mx[2], pz[q]) : mx[2];
        }
        const int kmv = (g.n_moves + n - 1) / n;
        const float e = (float)kmv * (delta * 1.000001f + 2e-7f) + 1e-5f;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            blo[ax] = fmaxf(mn[ax] - e, 0.0f);
            bhi[ax] = fminf(mx[ax] + e, g.w[ax]);
        }
    }

    // 2. translate into the cell's frame, keep what can reach the box;
    // K counts every kept sphere, the first kL go to the LDS column
    int K = 0;
    auto take = [&](const float4 &v, int q) {
        const int ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
        const float qx = frame(v.x, ox, g.w[0]);
        const float qy = frame(v.y, oy, g.w[1]);
        const float qz = frame(v.z, oz, g.w[2]);
        const float gx = fmaxf(fmaxf(blo[0] - qx, qx - bhi[0]), 0.0f);
        const float gy = fmaxf(fmaxf(blo[1] - qy, qy - bhi[1]), 0.0f);
        const float gz = fmaxf(fmaxf(blo[2] - qz, qz - bhi[2]), 0.0f);
        return make_float4(qx, qy, qz, (gx * gx + gy * gy) + gz * gz);
    };
    auto put = [&](const float4 &f, bool keep) {
        const int row = (keep && K < kL) ? K : kL;
        lx[row][lane] = f.x;
        ly[row][lane] = f.y;
        lz[row][lane] = f.z;
        K += keep ? 1 : 0;
    };
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const float4 f = take(v0[j][u], oq[j]);
            put(f, nmax > (uint32_t)u && nn[j] > (uint32_t)u && f.w < kReach2);
        }
    }
    // the rest slot by slot, while some lane of the wave has a cell with
    // more than i spheres.  These are raw buffer loads over the slot array:
    // a slot a lane does not need gets an offset past the buffer's end,
    // which the hardware's range check turns into zeros without a memory
    // access, so neither a branch nor a wasted cache line is spent on it.
    for (int i = kU; i < kCap; ++i) {
        if (__ballot(nmax > (uint32_t)i) == 0ull) break;
        float4 v[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const bool need = nmax > (uint32_t)i && nn[j] > (uint32_t)i;
            const int off = need ? (int)slot_of(g.C, cq[j], i) * (int)sizeof(float4) : kPastEnd;
            v[j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(slots, off, 0, 0));
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const float4 f = take(v[j], oq[j]);
            put(f, nmax > (uint32_t)i && nn[j] > (uint32_t)i && f.w < kReach2);
        }
    }
    const int KL = K < kL ? K : kL;
    // entries up to the wave's largest count in groups of four: far spheres
    // past each lane's own count
    int KLw = KL;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) KLw = max(KLw, __shfl_xor(KLw, o, 64));
    KLw = (KLw + 3) & ~3;
    for (int k = KL; k < KLw; ++k) {
        lx[k][lane] = kFar;
        ly[k][lane] = kFar;
        lz[k][lane] = kFar;
    }

    if (n > 0) {
        // rng.shuffle(c.particles): Fisher-Yates over the stored list on a
        // packed permutation (nibble q = source slot of list position q),
        // applied to the registers once; every lane of the group does the same
        uint32_t P = 0x76543210u;
        for (int k = 0; k < n - 1; ++k) {
            if (k > 0 && (k & 3) == 0)
                Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
            const int i = n - 1 - k;
            P = nib_swap(P, i, (int)bounded(word_of(Wsh, k & 3), (uint32_t)(i + 1)));
        }
        if (n > 1) {
            rperm(px, P);
            rperm(py, P);
            rperm(pz, P);
            if (has_tag) rperm(tg, P);
            if (has_acc) {
                rperm(ax, P);
                rperm(ay, P);
                rperm(az, P);
            }
        }
#pragma unroll
        for (int q = 1; q < kCap; ++q) {
            px[q] = q < n ? px[q] : kFar;
            py[q] = q < n ? py[q] : kFar;
            pz[q] = q < n ? pz[q] : kFar;
        }
    }
    // 3. the column, read once into registers (the loop bounds are the wave's)
    float rx[kL], ry[kL], rz[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) {
        rx[k] = k < KLw ? lx[k][lane] : kFar;
        ry[k] = k < KLw ? ly[k][lane] : kFar;
        rz[k] = k < KLw ? lz[k][lane] : kFar;
    }
    if (n > 0) {
        // the whole group takes this branch (n is the group's own count)
        const bool spill = K > kL;
        for (int t = 0; t < g.n_moves; ++t) {
            if (t > 0 && (t & 1) == 0) W = philox((uint32_t)c, s_lo, s_hi, (uint32_t)(t >> 1), k0, k1);
            float dx, dy, dz;
            displacement3((t & 1) ? W.z : W.x, (t & 1) ? W.w : W.y, delta, dx, dy, dz);
            const float xm = px[0] + dx;
            const float ym = py[0] + dy;
            const float zm = pz[0] + dz;
            bool ok = (xm > 0.0f) & (xm <= g.w[0]) & (ym > 0.0f) & (ym <= g.w[1]) &
                      (zm > 0.0f) & (zm <= g.w[2]);
#pragma unroll
            for (int q = 1; q < kCap; ++q) {
                const float ddx = xm - px[q];
                const float ddy = ym - py[q];
                const float ddz = zm - pz[q];
                ok = ok & !(pair_r2(ddx, ddy, ddz) < 1.0f);
            }
#pragma unroll
            for (int k = 0; k < kL; k += 4)
                if (k < KLw) ok = ok & !(min_r2_4(xm, ym, zm, rx + k, ry + k, rz + k) < 1.0f);
            if (spill && ok) ok = !overlap_from_memory(g, pos, count, cx, cy, cz, xm, ym, zm);
            ok = group_all<LPC>(ok);
            px[0] = ok ? xm : px[0];
            py[0] = ok ? ym : py[0];
            pz[0] = ok ? zm : pz[0];
            if (has_acc) {
                ax[0] = ok ? ax[0] + dx : ax[0];
                ay[0] = ok ? ay[0] + dy : ay[0];
                az[0] = ok ? az[0] + dz : az[0];
            }
            n_acc += (ok && h == 0) ? 1u : 0u;
            rrot(px, n);   // the identity for n = 1
            rrot(py, n);
            rrot(pz, n);
            if (has_tag) rrot(tg, n);
            if (has_acc) {
                rrot(ax, n);
                rrot(ay, n);
                rrot(az, n);
            }
        }
        if (h == 0) {
            n_trials = (unsigned)g.n_moves;
            // register entry q now holds list position (q + n_M) mod n
            const int r0 = g.n_moves % n;
#pragma unroll
            for (int q = 0; q < kCap; ++q) {
                if (q < n) {
                    int o = q + r0;
                    o = o >= n ? o - n : o;
                    const size_t so = slot_of(g.C, c, o);   // slot 0 carries the count
                    pos[so] = make_float4(px[q], py[q], pz[q], o == 0 ? __uint_as_float((uint32_t)n) : 0.0f);
                    if (has_tag && n > 1) tag[so] = tg[q];
                    if (has_acc) acc[so] = make_float4(ax[q], ay[q], az[q], 0.0f);
                }
            }
        }
    }
    // this workgroup's partials (one wave; the same entry in every launch)
    const unsigned bt = wave_sum_u32(n_trials);
    const unsigned ba = wave_sum_u32(n_acc);
    if (lane == 0 && tile < ntile && bt) {
        cnt[2 * tile] += (unsigned long long)bt;
        cnt[2 * tile + 1] += (unsigned long long)ba;
    }
}

// ------------------------------------------------------- brick sub-sweep
// The one-lane-per-cell form without accumulators.  A workgroup of 64
// lanes serves a brick of kBk^3 active cells of set Q; lane (lx, ly, lz)
// owns active cell (kBk bx + lx, ...).  The brick's region -- its cells and
// all their neighbours, kRg^3 cells with periodic indices -- is staged into
// LDS by coalesced loads that are all independent: the primary line of
// every cell (slots 0 and 1, the count in slot 0's fourth word), three
// rows of the region per load, and written out as one word per coordinate
// and slot (a far sphere where the slot is empty).  The region's cells with
// more than two spheres are compacted into a list of the brick, one entry
// per cell; each lane loads the slots 2..7 of one entry in a single round
// trip, issued before the lane fills its registers from LDS so that the
// two overlap, and hands them to the lists of the lanes whose
// neighbourhood holds that cell.  Each lane then holds the 52 staged slots
// of its 26 neighbour cells and its listed spheres in registers, translated
// into its frame (exactly -w, 0 or +w per axis), and runs its trials
// against all of them: no reach filter and no per-lane compaction.  A lane
// with more listed spheres than it holds, or a brick with more such cells
// than its list holds, tests every neighbour straight from memory instead
// (overlap_from_memory).  Every pair is tested with the same FP32
// operations as in the other forms, and a far sphere never overlaps, so the
// decisions are the same.
constexpr int kBk = 4;                     // active cells per brick side
constexpr int kRg = 2 * kBk + 1;           // region side, cells
constexpr int kRgC = kRg * kRg * kRg;      // region cells
constexpr int kOvLane = 8;                 // listed spheres a lane holds
constexpr int kOvCell = 128;               // listed cells with more than two spheres per brick

// LDS index of region cell (rx, ry, rz): per axis the even coordinates
// 0, 2, .., 8 come first (0..4), then the odd ones (5..8).  A lane's own
// cell has odd coordinates 2 l + 1 and its neighbours at offset -1 / +1
// have even ones 2 l / 2 l + 2, so the lanes of a wave, reading the same
// neighbour offset, read runs of consecutive words.
__device__ __forceinline__ constexpr int reg_axis(int r) { return (r >> 1) + 5 * (r & 1); }
__device__ __forceinline__ constexpr int reg_index(int rx, int ry, int rz)
{
    return reg_axis(rx) + kRg * (reg_axis(ry) + kRg * reg_axis(rz));
}

// x, y, z of the slot at byte offset off (a raw buffer load of 12 bytes).
__device__ __forceinline__ float3 slot_xyz(__amdgpu_buffer_rsrc_t r, int off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    return make_float3(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]));
}

template <bool TAG>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_subsweep3b(Geom3 g, Ctl3 *__restrict__ ctl, int par, float4 *__restrict__ pos,
             const uint32_t *__restrict__ count, uint32_t *__restrict__ tag,
             unsigned long long *__restrict__ cnt, int set, int nbrick, int per, int nbx, int nby)
{
    // slot planes [coordinate][slot][reg_index]; after the registers are
    // filled the same memory holds the per-lane lists [lane][k] (x, y, z)
    __shared__ float planes[6][kRgC];
    float(*sx)[kRgC] = planes, (*sy)[kRgC] = planes + 2, (*sz)[kRgC] = planes + 4;
    __shared__ uint32_t ov_lane[64];       // listed spheres per lane
    __shared__ int oc_cell[kOvCell];       // the region's cells with more than kPrim spheres
    __shared__ int oc_cn[kOvCell];         // their region code | count << 12
    static_assert(64 * kOvLane * 3 <= 6 * kRgC, "per-lane lists fit the slot planes");
    const int brick = xcd_tile(per);
    if (brick >= nbrick) return;           // a padding workgroup of the XCD-aligned grid
    const int lane = threadIdx.x;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int bz = brick / (nbx * nby), by = (brick / nbx) % nby, bx = brick % nbx;
    const int hx = g.m[0] >> 1, hy = g.m[1] >> 1, hz = g.m[2] >> 1;
    const int ix = kBk * bx + lx, iy = kBk * by + ly, iz = kBk * bz + lz;
    const bool live = ix < hx && iy < hy && iz < hz;
    const unsigned long long s = ctl->sweep_at[par];
    const uint32_t k0 = ctl->key0, k1 = ctl->key1;
    const float delta = ctl->delta;
    const uint32_t s_lo = (uint32_t)s, s_hi = (uint32_t)(s >> 32);
    int Q = set;
    if (Q < 0) Q = (int)((ctl->draw_at[par].order >> (4 * (-1 - set))) & 0xFu);
    const int qx = Q & 1, qy = (Q >> 1) & 1, qz = Q >> 2;
    // region origin (global cell coordinates of region cell (0, 0, 0)), may be -1
    const int ox0 = 2 * kBk * bx + qx - 1, oy0 = 2 * kBk * by + qy - 1, oz0 = 2 * kBk * bz + qz - 1;
    auto wrapc = [](int v, int m) {        // v in [-1, 3 m): the periodic image in [0, m)
        v = v < 0 ? v + m : v;
        v = v >= m ? v - m : v;
        return v >= m ? v - m : v;
    };
    ov_lane[lane] = 0u;
    const int cx = 2 * ix + qx, cy = 2 * iy + qy, cz = 2 * iz + qz;
    const int c = live ? (cz * g.m[1] + cy) * g.m[0] + cx : 0;
    constexpr bool has_tag = TAG;          // a compile-time variant: no registers without tags

    // 1. stage the region, three rows of kRg cells (kRg x 2 slots) per
    // step: lane l < 54 takes row j = l / 18 of the step's three and slot
    // l & 1 of region cell (l % 18) / 2, so a wave's load reads three runs of
    // consecutive 16-byte slots and each cache line once.  Lanes 54..63
    // repeat the loads of lanes 36..45 and write nothing.  Step t covers
    // rows ry = 3 (t % 3) + j, rz = t / 3.  Every load of this pass is
    // independent of the others.
    constexpr int kSt = kRg * kRg / 3;      // 27 steps
    const bool stg = lane < 54;
    const int ls = stg ? lane : lane - 18;
    const int jr = ls / 18, hs = ls & 1, rxs = (ls % 18) >> 1;
    const int gx = wrapc(ox0 + rxs, g.m[0]);
    int gy3[3], li3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gy3[a] = wrapc(oy0 + 3 * a + jr, g.m[1]);
        li3[a] = reg_axis(rxs) + kRg * reg_axis(3 * a + jr);
    }
    uint32_t cn[kSt];
    float4 v[kSt];
#pragma unroll
    for (int t = 0; t < kSt; ++t) {
        const int gz = wrapc(oz0 + t / 3, g.m[2]);
        const int cell = (gz * g.m[1] + gy3[t % 3]) * g.m[0] + gx;
        v[t] = pos[(size_t)cell * kPrim + hs];
    }
    // the cell's first random blocks, while the staging loads are in flight
    uint4 Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle, k0, k1);
    uint4 W = make_uint4(0, 0, 0, 0);
    if (g.n_moves > 0) W = philox((uint32_t)c, s_lo, s_hi, 0u, k0, k1);
#pragma unroll
    for (int t = 0; t < kSt; ++t) {
        // slot 0's fourth word is the cell's count; lane pairs (2 i, 2 i + 1)
        // hold slots 0 and 1 of one cell
        const uint32_t w0 = __float_as_uint(v[t].w);
        const uint32_t w1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)w0, 0xB1, 0xF, 0xF, false);
        cn[t] = hs == 0 ? w0 : w1;
    }
    const uint32_t n_raw = live ? count[c] : 0u;
    bool bad = n_raw > (uint32_t)kCap;
    // staging steps whose cell has more than kPrim spheres, the even steps
    // on the lane of slot 0 and the odd ones on the lane of slot 1; the
    // counts packed four bits each
    uint32_t ovm = 0u;
    uint32_t cpk[4] = {0u, 0u, 0u, 0u};
    if (stg) {
#pragma unroll
        for (int t = 0; t < kSt; ++t) {
            const uint32_t n = cn[t];
            const int li = li3[t % 3] + kRg * kRg * reg_axis(t / 3);
            bad |= n > (uint32_t)kCap;
            ovm |= ((t & 1) == hs && n > (uint32_t)kPrim) ? 1u << t : 0u;
            cpk[t >> 3] |= min(n, 15u) << (4 * (t & 7));
            const bool have = n > (uint32_t)hs;
            sx[hs][li] = have ? v[t].x : kFar;
            sy[hs][li] = have ? v[t].y : kFar;
            sz[hs][li] = have ? v[t].z : kFar;
        }
    }
    // 2. slots 2..7 of the staged cells that have them (more than kPrim
    // spheres): the cells are compacted into a list of the brick, one entry
    // per cell, and each lane then loads the slots of one entry per round, so
    // that one round trip serves the whole region.  The own cell's slots
    // 2..7 come in the same round trip.  A slot past the cell's count is a
    // raw buffer load past the buffer's end, which reads zeros without a
    // memory access.
    const __amdgpu_buffer_rsrc_t slots = __builtin_amdgcn_make_buffer_rsrc(
        (void *)pos, (short)0, (int)((unsigned)g.C * (unsigned)(kCap * sizeof(float4))), kBufferWord3);
    float px[kCap], py[kCap], pz[kCap];
#pragma unroll
    for (int q = 0; q < kCap; ++q) px[q] = py[q] = pz[q] = kFar;
    const int n = (live && __ballot(bad) == 0ull) ? (int)min(n_raw, (uint32_t)kCap) : 0;
    if (__ballot(bad) != 0ull) {
        // a cell above capacity: report it and leave the brick unchanged
        if (bad) atomicOr(&ctl->errword, kErrCapacity);
        ovm = 0u;
    }
    int noc = 0;                           // overflow cells of the region (wave-uniform)
    while (__ballot(ovm != 0u) != 0ull) {
        const bool have = ovm != 0u;
        const unsigned long long bal = __ballot(have);
        const int t = have ? __builtin_ctz(ovm) : 0;
        ovm &= have ? ovm - 1u : 0u;
        const int e = noc + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (have && e < kOvCell) {
            const int tw = t >> 3;
            const uint32_t pk = tw == 0 ? cpk[0] : (tw == 1 ? cpk[1] : (tw == 2 ? cpk[2] : cpk[3]));
            const uint32_t nc = min((pk >> (4 * (t & 7))) & 15u, (uint32_t)kCap);
            const int rz = t / 3, ry = 3 * (t - 3 * rz) + jr;
            oc_cell[e] = (wrapc(oz0 + rz, g.m[2]) * g.m[1] + wrapc(oy0 + ry, g.m[1])) * g.m[0] + gx;
            oc_cn[e] = (rxs | (ry << 4) | (rz << 8)) | (int)(nc << 12);
        }
        noc += __popcll(bal);
    }
    __syncthreads();
    const int ncl = noc < kOvCell ? noc : kOvCell;
    // the slots 2..7 of list entry e (zeros past its count), its region code
    // (12-byte loads: a fourth, unused register would be reallocated while the
    // load is in flight, and the compiler would wait for it)
    auto load_entry = [&](int e, float3 (&w)[kCap - kPrim], int &code, uint32_t &cnt) {
        const bool have = e < ncl;
        const int ce = have ? oc_cell[e] : 0;
        const int cc = have ? oc_cn[e] : 0;
        code = cc & 0xFFF;
        cnt = (uint32_t)cc >> 12;
#pragma unroll
        for (int q = kPrim; q < kCap; ++q) {
            if (q >= 4 && __ballot(cnt > (uint32_t)q) == 0ull) {
                w[q - kPrim] = make_float3(0.0f, 0.0f, 0.0f);
                continue;
            }
            const int off = cnt > (uint32_t)q ? (int)slot_of(g.C, ce, q) * (int)sizeof(float4) : kPastEnd;
            w[q - kPrim] = slot_xyz(slots, off);
        }
    };
    // the slots of an entry to the lists of the lanes whose neighbourhood
    // holds its cell (at most 8, the own lane excluded): per axis an even
    // region coordinate 2t neighbours lanes t - 1 (offset +1) and t (offset
    // -1), an odd one 2t + 1 only lane t (offset 0).  The lists take the slot
    // planes' memory, so this runs after the planes are read.
    float *lst = &planes[0][0];            // [lane][k][3]
    auto deal_entry = [&](const float3 (&w)[kCap - kPrim], int code, uint32_t cnt) {
        const int m = cnt > (uint32_t)kPrim ? (int)cnt - kPrim : 0;
        int mw = m;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mw = max(mw, __shfl_xor(mw, o, 64));
        if (mw == 0) return;
        const int r[3] = {code & 15, (code >> 4) & 15, code >> 8};
#pragma unroll
        for (int cmb = 0; cmb < 8; ++cmb) {
            int l[3], o[3];
            bool ok = m > 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int bit = (cmb >> d) & 1;
                if (r[d] & 1) {
                    l[d] = r[d] >> 1;
                    o[d] = 0;
                    ok = ok && bit == 0;
                } else {
                    l[d] = (r[d] >> 1) - 1 + bit;
                    o[d] = bit ? -1 : 1;
                }
                ok = ok && l[d] >= 0 && l[d] < kBk;
            }
            ok = ok && (o[0] | o[1] | o[2]) != 0;   // the own cell's spheres are the lane's own
            if (ok) {
                const int tl = l[0] + kBk * (l[1] + kBk * l[2]);
                const uint32_t k = atomicAdd(&ov_lane[tl], (uint32_t)m);
#pragma unroll
                for (int q = 0; q < kCap - kPrim; ++q) {
                    if (q < mw && q < m && k + (uint32_t)q < (uint32_t)kOvLane) {
                        float *dst = lst + (tl * kOvLane + (int)k + q) * 3;
                        dst[0] = frame(w[q].x, o[0], g.w[0]);
                        dst[1] = frame(w[q].y, o[1], g.w[1]);
                        dst[2] = frame(w[q].z, o[2], g.w[2]);
                    }
                }
            }
        }
    };
    if (__ballot(n > kPrim) != 0ull) {
#pragma unroll
        for (int q = kPrim; q < kCap; ++q) {
            const int off = n > q ? (int)slot_of(g.C, c, q) * (int)sizeof(float4) : kPastEnd;
            const float3 v = slot_xyz(slots, off);
            px[q] = v.x;
            py[q] = v.y;
            pz[q] = v.z;
        }
    }
    float3 w0[kCap - kPrim];
    int code0;
    uint32_t cnt0;
    load_entry(lane, w0, code0, cnt0);
    uint32_t tg[kCap];
#pragma unroll
    for (int q = 0; q < kCap; ++q) tg[q] = 0u;
    if (has_tag) {
#pragma unroll
        for (int q = 0; q < kCap; ++q)
            if (q < n) tg[q] = tag[slot_of(g.C, c, q)];
    }

    // 3. while those loads are in flight: the 26 neighbour cells' staged
    // slots, in this cell's frame
    const int rxo = 1 + 2 * lx, ryo = 1 + 2 * ly, rzo = 1 + 2 * lz;   // own region cell
    float nx[52], ny[52], nz[52];
#pragma unroll
    for (int j = 0; j < 26; ++j) {
        const int q = j < 13 ? j : j + 1;
        const int ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
        const int rn = reg_index(rxo + ox, ryo + oy, rzo + oz);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            nx[2 * j + u] = frame(sx[u][rn], ox, g.w[0]);
            ny[2 * j + u] = frame(sy[u][rn], oy, g.w[1]);
            nz[2 * j + u] = frame(sz[u][rn], oz, g.w[2]);
        }
    }
    const int ro = reg_index(rxo, ryo, rzo);
    px[0] = sx[0][ro];
    py[0] = sy[0][ro];
    pz[0] = sz[0][ro];
    px[1] = sx[1][ro];
    py[1] = sy[1][ro];
    pz[1] = sz[1][ro];
    deal_entry(w0, code0, cnt0);
    for (int r = 64; r < ncl; r += 64) {   // regions with more than 64 such cells
        float3 w1[kCap - kPrim];
        int code1;
        uint32_t cnt1;
        load_entry(r + lane, w1, code1, cnt1);
        deal_entry(w1, code1, cnt1);
    }
    __syncthreads();

    // 4. this lane's list; more than the list holds, or more listed cells than
    // the brick's list of cells holds, and the lane tests from memory
    const int kov = (int)ov_lane[lane];
    bool spill = noc > kOvCell || kov > kOvLane;
    float ex[kOvLane], ey[kOvLane], ez[kOvLane];
#pragma unroll
    for (int k = 0; k < kOvLane; ++k) {
        const float *src = lst + (lane * kOvLane + k) * 3;
        ex[k] = k < kov ? src[0] : kFar;
        ey[k] = k < kov ? src[1] : kFar;
        ez[k] = k < kov ? src[2] : kFar;
    }
    int kw = kov < kOvLane ? kov : kOvLane;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kw = max(kw, __shfl_xor(kw, o, 64));

    // 5. shuffle and trials; own entries at or past M = the wave's largest
    // count (2, 4 or 8) are far spheres or identities throughout, so the
    // phase is compiled for each M and the wave runs the smallest that fits
    int nw = n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nw = max(nw, __shfl_xor(nw, o, 64));
    unsigned n_trials = 0, n_acc = 0;
    auto phase = [&](auto Mc) {
        constexpr int M = decltype(Mc)::value;
        if (n == 0) return;
        // rng.shuffle(c.particles): Fisher-Yates on a packed permutation
        // (nibble q = source slot of list position q), applied once
        uint32_t P = 0x76543210u;
        for (int k = 0; k < n - 1; ++k) {
            if (k > 0 && (k & 3) == 0)
                Wsh = philox((uint32_t)c, s_lo, s_hi, kTagShuffle + (uint32_t)(k >> 2), k0, k1);
            const int i = n - 1 - k;
            P = nib_swap(P, i, (int)bounded(word_of(Wsh, k & 3), (uint32_t)(i + 1)));
        }
        if (n > 1) {
            rperm_m<M>(px, P);
            rperm_m<M>(py, P);
            rperm_m<M>(pz, P);
            if (has_tag) rperm_m<M>(tg, P);
        }
#pragma unroll
        for (int q = 1; q < M; ++q) {
            px[q] = q < n ? px[q] : kFar;
            py[q] = q < n ? py[q] : kFar;
            pz[q] = q < n ? pz[q] : kFar;
        }
        for (int t = 0; t < g.n_moves; ++t) {
            if (t > 0 && (t & 1) == 0) W = philox((uint32_t)c, s_lo, s_hi, (uint32_t)(t >> 1), k0, k1);
            float dx, dy, dz;
            displacement3((t & 1) ? W.z : W.x, (t & 1) ? W.w : W.y, delta, dx, dy, dz);
            const float xm = px[0] + dx;
            const float ym = py[0] + dy;
            const float zm = pz[0] + dz;
            bool ok = (xm > 0.0f) & (xm <= g.w[0]) & (ym > 0.0f) & (ym <= g.w[1]) &
                      (zm > 0.0f) & (zm <= g.w[2]);
#pragma unroll
            for (int q = 1; q < M; ++q) {
                const float ddx = xm - px[q];
                const float ddy = ym - py[q];
                const float ddz = zm - pz[q];
                ok = ok & !(pair_r2(ddx, ddy, ddz) < 1.0f);
            }
#pragma unroll
            for (int k = 0; k < 52; k += 4)
                ok = ok & !(min_r2_4(xm, ym, zm, nx + k, ny + k, nz + k) < 1.0f);
#pragma unroll
            for (int k = 0; k < kOvLane; k += 4)
                if (k < kw) ok = ok & !(min_r2_4(xm, ym, zm, ex + k, ey + k, ez + k) < 1.0f);
            if (spill && ok) ok = !overlap_from_memory(g, pos, count, cx, cy, cz, xm, ym, zm);
            px[0] = ok ? xm : px[0];
            py[0] = ok ? ym : py[0];
            pz[0] = ok ? zm : pz[0];
            n_acc += ok ? 1u : 0u;
            rrot_m<M>(px, n);   // the identity for n = 1
            rrot_m<M>(py, n);
            rrot_m<M>(pz, n);
            if (has_tag) rrot_m<M>(tg, n);
        }
        n_trials = (unsigned)g.n_moves;
        // register entry q now holds list position (q + n_M) mod n
        const int r0 = g.n_moves % n;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            if (q < n) {
                int o = q + r0;
                o = o >= n ? o - n : o;
                const size_t so = slot_of(g.C, c, o);   // slot 0 carries the count
                pos[so] = make_float4(px[q], py[q], pz[q], o == 0 ? __uint_as_float((uint32_t)n) : 0.0f);
                if (has_tag && n > 1) tag[so] = tg[q];
            }
        }
    };
    if (nw <= 2)
        phase(std::integral_constant<int, 2>{});
    else if (nw <= 4)
        phase(std::integral_constant<int, 4>{});
    else
        phase(std::integral_constant<int, kCap>{});
    // this workgroup's partials (one wave; the same entry in every launch)
    const unsigned bt = wave_sum_u32(n_trials);
    const unsigned ba = wave_sum_u32(n_acc);
    if (lane == 0 && bt) {
        cnt[2 * brick] += (unsigned long long)bt;
        cnt[2 * brick + 1] += (unsigned long long)ba;
    }
}

// Add the partials into the control block and clear them (one workgroup).
__global__ void __launch_bounds__(256) k_fold3(Ctl3 *ctl, unsigned long long *cnt, int groups)
{
    __shared__ unsigned long long sh[8];
    unsigned long long tr = 0, ac = 0;
    for (int i = threadIdx.x; i < groups; i += blockDim.x) {
        tr += cnt[2 * i];
        ac += cnt[2 * i + 1];
        cnt[2 * i] = 0ull;
        cnt[2 * i + 1] = 0ull;
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
        ctl->trials += sh[0] + sh[1] + sh[2] + sh[3];
        ctl->accepts += sh[4] + sh[5] + sh[6] + sh[7];
    }
}

// ----------------------------------------------------------------- rebin
// Alg. 4 in d = 3 on the slot layout: new cell c holds the stayers of old c
// followed by the spheres of the old neighbour in direction f that move in,
// both in old slot order.  One thread per cell; the counts and the primary
// lines of both cells are loaded in one round trip, the overflow slots only
// where a count needs them.  Slot 0 of every new cell is written, with the
// new count in its fourth word.  The first workgroup writes
// the sweep slot of the half it writes: the next sweep and its draws when
// the shift is the sweep's own, else a copy of the current slot.
struct Rebin3Args {
    Geom3 g;
    Ctl3 *ctl;
    const float4 *pos;
    const uint32_t *count;
    const uint32_t *tag;
    const float4 *acc;
    float4 *pos_out;
    uint32_t *count_out;
    uint32_t *tag_out;
    float4 *acc_out;
    int par;
    int f;        // >= 0 explicit; < 0 the sweep's own
    float d;
    int ntile;
    int per;
};

__global__ void __launch_bounds__(kTile) k_rebin3(Rebin3Args a)
{
    const int tile = xcd_tile(a.per);
    if (tile >= a.ntile) return;
    const Geom3 &g = a.g;
    Ctl3 *ctl = a.ctl;
    int f = a.f;
    float d = a.d;
    if (f < 0) {
        f = ctl->draw_at[a.par].f;
        d = ctl->draw_at[a.par].d;
    }
    const int ax = f >> 1;
    const bool minus = (f & 1) == 0;   // +x, +y, +z: t = v - d, leavers come from cell + 1
    const float w = g.w[ax];
    const float sw = minus ? w : -w;
    const int c = tile * kTile + (int)threadIdx.x;
    if (c < g.C) {
        const int cx = c % g.m[0], cy = (c / g.m[0]) % g.m[1], cz = c / (g.m[0] * g.m[1]);
        int n3[3] = {cx, cy, cz};
        const int cc = ax == 0 ? cx : (ax == 1 ? cy : cz);
        const int mm = g.m[ax];
        const int nv = minus ? (cc == mm - 1 ? 0 : cc + 1) : (cc == 0 ? mm - 1 : cc - 1);
        if (ax == 0) n3[0] = nv;
        else if (ax == 1) n3[1] = nv;
        else n3[2] = nv;
        const int nc = (n3[2] * g.m[1] + n3[1]) * g.m[0] + n3[0];
        int no = (int)a.count[c];
        int nn = (int)a.count[nc];
        // both primary lines with the counts; the overflow slots only for
        // cells with more than kPrim spheres
        float4 own[kCap], nb[kCap];
#pragma unroll
        for (int i = 0; i < kCap; ++i) {
            own[i] = nb[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (i < kPrim) {
                own[i] = a.pos[slot_of(g.C, c, i)];
                nb[i] = a.pos[slot_of(g.C, nc, i)];
            }
        }
        if (no > kPrim || nn > kPrim) {
#pragma unroll
            for (int i = kPrim; i < kCap; ++i) {
                if (i < no) own[i] = a.pos[slot_of(g.C, c, i)];
                if (i < nn) nb[i] = a.pos[slot_of(g.C, nc, i)];
            }
        }
        if (no > kCap || nn > kCap) {
            atomicOr(&ctl->errword, kErrCapacity);
            no = min(no, kCap);
            nn = min(nn, kCap);
        }
        unsigned stay = 0, leave = 0;
        float to[kCap], tn[kCap];
#pragma unroll
        for (int i = 0; i < kCap; ++i) {
            const float vo = ax == 0 ? own[i].x : (ax == 1 ? own[i].y : own[i].z);
            const float vn = ax == 0 ? nb[i].x : (ax == 1 ? nb[i].y : nb[i].z);
            to[i] = minus ? vo - d : vo + d;
            tn[i] = minus ? vn - d : vn + d;
            if (i < no && to[i] > 0.0f && to[i] <= w) stay |= 1u << i;
            if (i < nn && !(tn[i] > 0.0f && tn[i] <= w)) leave |= 1u << i;
        }
        const unsigned k = (unsigned)(__popc(stay) + __popc(leave));
        if (k > (unsigned)kCap) atomicOr(&ctl->errword, kErrCapacity);
        const unsigned kc = k > (unsigned)kCap ? (unsigned)kCap : k;
        a.count_out[c] = kc;
        if (kc == 0u) a.pos_out[slot_of(g.C, c, 0)] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const bool has_tag = a.tag != nullptr;
        int o = 0;   // next slot of the new list (never past the cell's 8)
#pragma unroll
        for (int i = 0; i < kCap; ++i) {
            if ((stay & (1u << i)) && o < kCap) {
                float4 v = own[i];
                if (ax == 0) v.x = to[i];
                else if (ax == 1) v.y = to[i];
                else v.z = to[i];
                v.w = o == 0 ? __uint_as_float(kc) : 0.0f;
                a.pos_out[slot_of(g.C, c, o)] = v;
                if (has_tag) a.tag_out[slot_of(g.C, c, o)] = a.tag[slot_of(g.C, c, i)];
                if (a.acc) a.acc_out[slot_of(g.C, c, o)] = a.acc[slot_of(g.C, c, i)];
            }
            o += (stay >> i) & 1u;
        }
#pragma unroll
        for (int i = 0; i < kCap; ++i) {
            if ((leave & (1u << i)) && o < kCap) {
                float4 v = nb[i];
                const float t2 = tn[i] + sw;
                if (ax == 0) v.x = t2;
                else if (ax == 1) v.y = t2;
                else v.z = t2;
                v.w = o == 0 ? __uint_as_float(kc) : 0.0f;
                a.pos_out[slot_of(g.C, c, o)] = v;
                if (has_tag) a.tag_out[slot_of(g.C, c, o)] = a.tag[slot_of(g.C, nc, i)];
                if (a.acc) a.acc_out[slot_of(g.C, c, o)] = a.acc[slot_of(g.C, nc, i)];
            }
            o += (leave >> i) & 1u;
        }
    }
    if (tile == 0 && threadIdx.x == 0) {
        const unsigned long long s = ctl->sweep_at[a.par];
        if (a.f < 0) {
            store_draws3(ctl, a.par ^ 1, s + 1ull, g);
        } else {
            ctl->sweep_at[a.par ^ 1] = s;
            ctl->draw_at[a.par ^ 1] = ctl->draw_at[a.par];
        }
    }
}

// ---------------------------------------------------------- control block
__global__ void __launch_bounds__(256)
k_ctl_reset3(Geom3 g, Ctl3 *ctl, unsigned long long sweep, unsigned int key0, unsigned int key1,
             float delta)
{
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0ull;
    if (threadIdx.x == 0) {
        ctl->trials = ctl->accepts = 0ull;
        ctl->win_trials = ctl->win_accepts = 0ull;
        ctl->key0 = key0;
        ctl->key1 = key1;
        ctl->delta = delta;
        ctl->errword = 0u;
        ctl->hist_samples = 0ull;
        for (int k = 0; k < 4; ++k) ctl->fit[k] = 0.0;
        ctl->overlaps = 0;
        store_draws3(ctl, 0, sweep, g);
        ctl->sweep_at[1] = ctl->sweep_at[0];
        ctl->draw_at[1] = ctl->draw_at[0];
        ctl->draw_at[0].pad = ctl->draw_at[1].pad = 0u;
    }
}

__global__ void k_set_delta3(Ctl3 *ctl, float delta) { ctl->delta = delta; }

// The plain tuner between equilibration windows: with a = accepts / trials
// of the window, delta <- delta clamp(a / 0.3, 0.5, 2), clamped to
// [1e-3, min(w) / 2], in FP64 and rounded once to FP32 (the same rule as
// for disks, with the smallest of three widths).
__global__ void k_tune3(Geom3 g, Ctl3 *ctl, int apply)
{
    const unsigned long long tr = ctl->trials - ctl->win_trials;
    const unsigned long long a = ctl->accepts - ctl->win_accepts;
    if (apply && tr > 0) {
        double q = ((double)a / (double)tr) / 0.3;
        if (q < 0.5) q = 0.5;
        if (q > 2.0) q = 2.0;
        double nd = (double)ctl->delta * q;
        const float wmin = fminf(g.w[0], fminf(g.w[1], g.w[2]));
        const double hi = 0.5 * (double)wmin;
        if (nd < 1e-3) nd = 1e-3;
        if (nd > hi) nd = hi;
        ctl->delta = (float)nd;
    }
    ctl->win_trials = ctl->trials;
    ctl->win_accepts = ctl->accepts;
}

// ------------------------------------------------------ pair histogram
// Ordered pairs (k, j != k) with r^2 in k's frame, translations o w with
// o in [-R, R] per axis (R = 2 where w < 1.02), binned on
// E_b = (float)((1 + b 1e-4)^2).  One thread per cell.
__global__ void __launch_bounds__(kTile)
k_pair_hist3(Geom3 g, Ctl3 *ctl, const float4 *__restrict__ pos,
             const uint32_t *__restrict__ count, int ntile, int per)
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
    const double rmax = 1.0 + kHistBins * 1e-4;
    int Rr[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) Rr[q] = (double)g.w[q] >= rmax ? 1 : 2;
    const int c = tile * kTile + (int)threadIdx.x;
    if (tile < ntile && c < g.C) {
        const int cx = c % g.m[0], cy = (c / g.m[0]) % g.m[1], cz = c / (g.m[0] * g.m[1]);
        const float e0 = E[0], eN = E[kHistBins];
        const uint32_t nk = min(count[c], (uint32_t)kCap);
        for (uint32_t k = 0; k < nk; ++k) {
            const float4 pk = pos[slot_of(g.C, c, (int)k)];
            for (int oz = -Rr[2]; oz <= Rr[2]; ++oz) {
                const int ncz = (cz + oz + 2 * g.m[2]) % g.m[2];
                const float tz = (float)oz * g.w[2];
                for (int oy = -Rr[1]; oy <= Rr[1]; ++oy) {
                    const int ncy = (cy + oy + 2 * g.m[1]) % g.m[1];
                    const float ty = (float)oy * g.w[1];
                    for (int ox = -Rr[0]; ox <= Rr[0]; ++ox) {
                        const int ncx = (cx + ox + 2 * g.m[0]) % g.m[0];
                        const float tx = (float)ox * g.w[0];
                        const int nc = (ncz * g.m[1] + ncy) * g.m[0] + ncx;
                        for (uint32_t j = 0, je = min(count[nc], (uint32_t)kCap); j < je; ++j) {
                            if (nc == c && j == k) continue;
                            const float4 v = pos[slot_of(g.C, nc, (int)j)];
                            const float ddx = pk.x - (v.x + tx);
                            const float ddy = pk.y - (v.y + ty);
                            const float ddz = pk.z - (v.z + tz);
                            const float r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
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
    }
    __syncthreads();
    if (tile < ntile) {
        for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
            if (H[i]) atomicAdd(&ctl->hist[i], (unsigned long long)H[i]);
        if (tile == 0 && threadIdx.x == 0) atomicAdd(&ctl->hist_samples, 1ull);
    }
}

__global__ void k_hist_reset3(Ctl3 *ctl)
{
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0ull;
    if (threadIdx.x == 0) ctl->hist_samples = 0ull;
}

// ------------------------------------------------------ contact fit (FP64)
// g(R_i) = n_i / (S N rho 4 pi R_i^2 dr) at the volume-weighted shell radii
// R_i = 3/4 (r1^4 - r0^4) / (r1^3 - r0^3); unweighted least squares of a
// degree-5 polynomial in (R - 1)/0.02 by Householder QR; the contact
// theorem in 3D, beta P = rho (1 + 2 pi/3 rho g(sigma+)).
__global__ void __launch_bounds__(256) k_pressure_fit3(Geom3 g, Ctl3 *ctl)
{
    constexpr int NB = kHistBins, NC = 6;
    __shared__ double A[NB][NC];
    __shared__ double y[NB];
    __shared__ double v[NB];
    const unsigned long long S = ctl->hist_samples;
    const double vol = ((double)g.m[0] * (double)g.w[0]) * ((double)g.m[1] * (double)g.w[1]) *
                       ((double)g.m[2] * (double)g.w[2]);
    const double rho = (double)g.N / vol;
    const double dr = 1e-4, cfit = 0.02, pi = 3.14159265358979323846;
    for (int i = threadIdx.x; i < NB; i += blockDim.x) {
        const double r0 = 1.0 + (double)i * dr;
        const double r1 = 1.0 + (double)(i + 1) * dr;
        const double r02 = r0 * r0, r12 = r1 * r1;
        const double Ri = 0.75 * (r12 * r12 - r02 * r02) / (r12 * r1 - r02 * r0);
        const double n = (double)ctl->hist[i] / (double)(S ? S : 1ull);
        y[i] = n / ((double)g.N * rho * 4.0 * pi * Ri * Ri * dr);
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
    ctl->fit[0] = rho * (1.0 + (2.0 * pi / 3.0) * rho * coef[0]);
    ctl->fit[1] = coef[0];
    ctl->fit[2] = rho;
    ctl->fit[3] = 1.0;
}

// ------------------------------------------------------ overlap count
// Ordered pairs with r^2 < 1 - 2^-20 in either sphere's frame (the trial
// moves test r^2 < 1 in the mover's frame; seen from the partner the same
// pair may round a few ulp below 1, and each rebin re-expresses a
// coordinate with one rounding while neither sphere moves).
constexpr float kOverlapR2 = 1.0f - 0x1p-20f;

__global__ void __launch_bounds__(kTile)
k_count_overlaps3(Geom3 g, Ctl3 *ctl, const float4 *__restrict__ pos,
                  const uint32_t *__restrict__ count, int ntile, int per)
{
    __shared__ unsigned red[4];
    const int tile = xcd_tile(per);
    const int c = tile * kTile + (int)threadIdx.x;
    unsigned bad = 0;
    if (tile < ntile && c < g.C) {
        const int cx = c % g.m[0], cy = (c / g.m[0]) % g.m[1], cz = c / (g.m[0] * g.m[1]);
        const uint32_t nk = min(count[c], (uint32_t)kCap);
        for (uint32_t k = 0; k < nk; ++k) {
            const float4 pk = pos[slot_of(g.C, c, (int)k)];
            for (int q = 0; q < 27; ++q) {
                const int ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
                const int nx = (cx + ox + g.m[0]) % g.m[0];
                const int ny = (cy + oy + g.m[1]) % g.m[1];
                const int nz = (cz + oz + g.m[2]) % g.m[2];
                const int nc = (nz * g.m[1] + ny) * g.m[0] + nx;
                for (uint32_t j = 0, je = min(count[nc], (uint32_t)kCap); j < je; ++j) {
                    if (nc == c && j == k) continue;
                    const float4 v = pos[slot_of(g.C, nc, (int)j)];
                    const float ddx = pk.x - frame(v.x, ox, g.w[0]);
                    const float ddy = pk.y - frame(v.y, oy, g.w[1]);
                    const float ddz = pk.z - frame(v.z, oz, g.w[2]);
                    bad += ((ddx * ddx + ddy * ddy) + ddz * ddz < kOverlapR2) ? 1u : 0u;
                }
            }
        }
    }
    bad = wave_sum_u32(bad);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0 && tile < ntile) {
        const unsigned tot = red[0] + red[1] + red[2] + red[3];
        if (tot) atomicAdd((unsigned long long *)&ctl->overlaps, (unsigned long long)tot);
    }
}

__global__ void k_overlaps_reset3(Ctl3 *ctl) { ctl->overlaps = 0; }

// ------------------------------------------------------------------ MSD
// Mean |acc|^2 over the N spheres, FP64, in a fixed order: one partial per
// tile of kTile cells (its lanes' sums folded in a fixed tree), then one
// thread adds the partials in tile order.
__global__ void __launch_bounds__(kTile)
k_msd3_partial(Geom3 g, const float4 *__restrict__ acc, const uint32_t *__restrict__ count,
               double *__restrict__ part)
{
    __shared__ double sh[kTile];
    const int c = blockIdx.x * kTile + (int)threadIdx.x;
    double v = 0.0;
    if (c < g.C) {
        const uint32_t n = min(count[c], (uint32_t)kCap);
        for (uint32_t i = 0; i < n; ++i) {
            const float4 a = acc[slot_of(g.C, c, (int)i)];
            v += ((double)a.x * a.x + (double)a.y * a.y) + (double)a.z * a.z;
        }
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kTile / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_msd3_final(Geom3 g, Ctl3 *ctl, const double *part, int nb)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    ctl->msd = g.N > 0 ? s / (double)g.N : 0.0;
}

__global__ void k_zero4(float4 *p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

// ---------------------------------------------------------------- launches
hipError_t launch_subsweep3(const Geom3 &g, Ctl3 *ctl, int par, float4 *pos,
                            const uint32_t *count, uint32_t *tag, float4 *acc,
                            unsigned long long *cnt, int set, int lanes, hipStream_t st)
{
    const int ntile = subsweep_tiles(g, lanes);
    const int grid = xcd_groups(ntile);
#define SPH_SUB(L, A)                                                                         \
    hipLaunchKernelGGL((k_subsweep3<L, A>), dim3(grid), dim3(kSubBlock), 0, st, g, ctl, par, pos, \
                       count, tag, acc, cnt, set, ntile, grid / 8)
    const bool a = acc != nullptr;
    if (lanes == 4) {
        if (a) SPH_SUB(4, true); else SPH_SUB(4, false);
    } else if (lanes == 2) {
        if (a) SPH_SUB(2, true); else SPH_SUB(2, false);
    } else {
        // one lane per cell: the brick form, or with accumulators the
        // per-lane form (the brick's registers have no room for them)
        const int nbx = brick_count(g.m[0]), nby = brick_count(g.m[1]), nbz = brick_count(g.m[2]);
        const int nbrick = nbx * nby * nbz;
        const int bgrid = xcd_groups(nbrick);
        if (a)
            SPH_SUB(1, true);
        else if (tag)
            hipLaunchKernelGGL(k_subsweep3b<true>, dim3(bgrid), dim3(64), 0, st, g, ctl, par, pos,
                               count, tag, cnt, set, nbrick, bgrid / 8, nbx, nby);
        else
            hipLaunchKernelGGL(k_subsweep3b<false>, dim3(bgrid), dim3(64), 0, st, g, ctl, par, pos,
                               count, tag, cnt, set, nbrick, bgrid / 8, nbx, nby);
    }
#undef SPH_SUB
    return hipGetLastError();
}

hipError_t launch_fold3(const Geom3 &g, Ctl3 *ctl, unsigned long long *cnt, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold3, dim3(1), dim3(256), 0, st, ctl, cnt, subsweep_groups(g));
    return hipGetLastError();
}

hipError_t launch_rebin3(const Geom3 &g, Ctl3 *ctl, int par, const float4 *pos,
                         const uint32_t *count, const uint32_t *tag, const float4 *acc,
                         float4 *pos_out, uint32_t *count_out, uint32_t *tag_out, float4 *acc_out,
                         int f, float d, hipStream_t st)
{
    Rebin3Args a;
    a.g = g;
    a.ctl = ctl;
    a.pos = pos;
    a.count = count;
    a.tag = tag;
    a.acc = acc;
    a.pos_out = pos_out;
    a.count_out = count_out;
    a.tag_out = tag_out;
    a.acc_out = acc_out;
    a.par = par;
    a.f = f;
    a.d = d;
    a.ntile = (g.C + kTile - 1) / kTile;
    const int grid = xcd_groups(a.ntile);
    a.per = grid / 8;
    hipLaunchKernelGGL(k_rebin3, dim3(grid), dim3(kTile), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_msd3(const Geom3 &g, Ctl3 *ctl, const float4 *acc, const uint32_t *count,
                       double *part, hipStream_t st)
{
    const int nb = (g.C + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_msd3_partial, dim3(nb), dim3(kTile), 0, st, g, acc, count, part);
    hipLaunchKernelGGL(k_msd3_final, dim3(1), dim3(64), 0, st, g, ctl, part, nb);
    return hipGetLastError();
}

hipError_t launch_zero4(float4 *p, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_ctl_reset3(const Geom3 &g, Ctl3 *ctl, unsigned long long sweep,
                             unsigned int key0, unsigned int key1, float delta, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctl_reset3, dim3(1), dim3(256), 0, st, g, ctl, sweep, key0, key1, delta);
    return hipGetLastError();
}

hipError_t launch_set_delta3(Ctl3 *ctl, float delta, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_delta3, dim3(1), dim3(1), 0, st, ctl, delta);
    return hipGetLastError();
}

hipError_t launch_tune3(const Geom3 &g, Ctl3 *ctl, int apply, hipStream_t st)
{
    hipLaunchKernelGGL(k_tune3, dim3(1), dim3(1), 0, st, g, ctl, apply);
    return hipGetLastError();
}

hipError_t launch_pair_hist3(const Geom3 &g, Ctl3 *ctl, const float4 *pos, const uint32_t *count,
                             int reset, hipStream_t st)
{
    if (reset) hipLaunchKernelGGL(k_hist_reset3, dim3(1), dim3(256), 0, st, ctl);
    const int ntile = (g.C + kTile - 1) / kTile;
    const int grid = xcd_groups(ntile);
    hipLaunchKernelGGL(k_pair_hist3, dim3(grid), dim3(kTile), 0, st, g, ctl, pos, count, ntile,
                       grid / 8);
    return hipGetLastError();
}

hipError_t launch_pressure_fit3(const Geom3 &g, Ctl3 *ctl, hipStream_t st)
{
    hipLaunchKernelGGL(k_pressure_fit3, dim3(1), dim3(256), 0, st, g, ctl);
    return hipGetLastError();
}

hipError_t launch_count_overlaps3(const Geom3 &g, Ctl3 *ctl, const float4 *pos,
                                  const uint32_t *count, hipStream_t st)
{
    hipLaunchKernelGGL(k_overlaps_reset3, dim3(1), dim3(1), 0, st, ctl);
    const int ntile = (g.C + kTile - 1) / kTile;
    const int grid = xcd_groups(ntile);
    hipLaunchKernelGGL(k_count_overlaps3, dim3(grid), dim3(kTile), 0, st, g, ctl, pos, count,
                       ntile, grid / 8);
    return hipGetLastError();
}

}  // namespace sph
}  // namespace mpmc
