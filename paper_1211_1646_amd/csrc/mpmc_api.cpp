// Host side of libmpmc.so: the C ABI declared in include/mpmc.h.
//
// Validates arguments and geometry, builds the initial lattices, owns no
// device memory (the caller's buffers are used through non-owning pointers),
// and enqueues the kernels of mpmc_kernels.hip on the caller's stream.  A
// handle holds R >= 1 replicas laid out back to back (a single system is
// R = 1); every kernel launch covers all of them.  Long runs of sweeps are
// captured once into hipGraphs of a fixed, even number of sweeps (the
// ping-pong buffers return to the same half after each graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpmc.h"
#include "mpmc_internal.h"

using mpmc::Ctl;
using mpmc::Geom;
using mpmc::Rep;

namespace {

thread_local std::string g_last_error;

mpmc_status fail(mpmc_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define MPMC_HIP(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(MPMC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr int kGraphSweeps = 16;   // sweeps per captured graph (even)
constexpr int kMaxReplicas = 65535;

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Largest number of non-overlapping unit-diameter disk centres in a square of
// side w (Fig. 3 for five; optimal packings of six, seven and eight points),
// with a 1e-5 relative margin for the FP32 overlap metric.
int capacity_of_width(double w)
{
    const double m = 1.0 - 1e-5;
    if (w < std::sqrt(2.0) * m) return 4;
    if (w < 6.0 / std::sqrt(13.0) * m) return 5;
    if (w < (2.0 + std::sqrt(3.0)) / 2.0 * m) return 6;
    if (w < (std::sqrt(6.0) + std::sqrt(2.0)) / 2.0 * m) return 7;
    return -1;
}

// Even cell count along an axis of length L.
int cells_along(double L, int requested, double w_min, double w_max)
{
    if (requested > 0) return requested;
    if (w_max > 0.0) {   // smallest even m with L/m < w_max
        int m = 2;
        const int guess = 2 * (int)std::floor(L / (2.0 * w_max));
        if (guess > 2) m = guess;
        while (L / (double)m >= w_max) m += 2;
        while (m > 2 && L / (double)(m - 2) < w_max) m -= 2;
        return m;
    }
    // largest even m with L/m >= w_min
    int m = 2 * (int)std::floor(L / (2.0 * w_min)) + 2;
    while (m > 0 && L / (double)m < w_min) m -= 2;
    return m;
}

struct Lattice {
    double a = 0, h = 0, Lx = 0, Ly = 0;
};

// Triangular lattice of nx x ny sites at packing fraction phi: area
// A = N pi / (4 phi), A = nx ny a^2 sqrt(3)/2, rows h = a sqrt(3)/2 apart.
Lattice lattice_of(int nx, int ny, double phi)
{
    Lattice L;
    const double N = (double)nx * (double)ny;
    const double A = N * kPi / (4.0 * phi);
    L.a = std::sqrt(2.0 * A / (std::sqrt(3.0) * N));
    L.h = L.a * std::sqrt(3.0) / 2.0;
    L.Lx = (double)nx * L.a;
    L.Ly = (double)ny * L.h;
    return L;
}

mpmc_status derive_geometry(const mpmc_params *p, mpmc_geometry *g)
{
    if (!p || !g) return fail(MPMC_EINVAL, "null argument");
    std::memset(g, 0, sizeof(*g));
    int mx, my;
    float wx, wy;
    if (p->lattice_nx > 0) {
        if (p->lattice_ny < 2 || (p->lattice_ny & 1))
            return fail(MPMC_EINVAL, "lattice_ny must be even and >= 2");
        if (!(p->phi > 0.0 && p->phi < 0.9)) return fail(MPMC_EINVAL, "phi must lie in (0, 0.9)");
        const Lattice L = lattice_of(p->lattice_nx, p->lattice_ny, p->phi);
        const double w_min = p->w_min > 0.0 ? p->w_min : 1.0;
        mx = cells_along(L.Lx, p->cells_x, w_min, p->w_max);
        my = cells_along(L.Ly, p->cells_y, w_min, p->w_max);
        if (mx < 4 || my < 4 || (mx & 1) || (my & 1))
            return fail(MPMC_EGEOM, "cell grid must be even and at least 4 x 4");
        wx = (float)(L.Lx / (double)mx);
        wy = (float)(L.Ly / (double)my);
        g->n_particles = (int64_t)p->lattice_nx * p->lattice_ny;
    } else {
        mx = p->cells_x;
        my = p->cells_y;
        wx = p->cell_w_x;
        wy = p->cell_w_y;
        if (mx < 4 || my < 4 || (mx & 1) || (my & 1))
            return fail(MPMC_EGEOM, "cell grid must be even and at least 4 x 4");
        if (p->n_particles < 0) return fail(MPMC_EINVAL, "n_particles < 0");
        g->n_particles = p->n_particles;
    }
    if (!(wx >= 1.0f && wy >= 1.0f)) return fail(MPMC_EGEOM, "cell width below sigma = 1");
    const int cap = capacity_of_width(std::max((double)wx, (double)wy));
    if (cap < 0) return fail(MPMC_EGEOM, "cell width too large (capacity above 7)");
    if ((long long)mx * my > 0x7FFFFFF0LL) return fail(MPMC_EGEOM, "too many cells");
    if (g->n_particles > (long long)cap * mx * my) return fail(MPMC_EGEOM, "more disks than cells can hold");
    g->cells_x = mx;
    g->cells_y = my;
    g->w_x = wx;
    g->w_y = wy;
    g->capacity = cap;
    g->box_x = (double)mx * (double)wx;
    g->box_y = (double)my * (double)wy;
    g->density = (double)g->n_particles / (g->box_x * g->box_y);
    return MPMC_OK;
}

// Flags that change only the chain, not the buffers: may differ between replicas.
constexpr uint32_t kChainFlags = MPMC_FLAG_DISK | MPMC_FLAG_NO_PARTICLE_SHUFFLE |
                                 MPMC_FLAG_NO_SET_SHUFFLE | MPMC_FLAG_LEAVE | MPMC_FLAG_LEAVE_ONCE;

mpmc_status check_params(const mpmc_params *p, const mpmc_geometry &g)
{
    if (!(p->delta > 0.0f) || p->delta > 0.5f * std::min(g.w_x, g.w_y))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    if (p->n_moves < 0 || p->n_moves > (1 << 20)) return fail(MPMC_EINVAL, "n_moves out of range");
    if (p->flags & ~(MPMC_FLAG_ACC | MPMC_FLAG_TAG | MPMC_FLAG_ACCEPT_LOG | kChainFlags))
        return fail(MPMC_EINVAL, "unknown flag");
    return MPMC_OK;
}

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

// Placement of the replicas: cells padded to whole rebin tiles, active slots
// to whole active chunks, disks back to back.
struct Layout {
    std::vector<mpmc_geometry> geo;
    std::vector<Rep> reps;
    long long N = 0, cells = 0, active = 0;
    long long ftiles = 0;   // fused-sweep tiles, all replicas, at the chosen shape
    long long ftiles_max = 0;   // ... at the smallest shape (sizes the tile table)
    int ftile = 0;          // largest tile side the buffer flags allow
    int ftx = 0, fty = 0;   // the chosen shape
    int cap = 0;
};

// The fused sweep's tile shape (tx, ty even, kFusedMinTile..ftile) for a
// device of `cus` compute units, two workgroups resident per CU: the sweep
// is VALU-bound, so its time is about the busiest CU's work, the tiles it
// runs times the updates of one tile (the four sub-sweeps' boxes, the
// interior grown by 3.5, 2.5, 1.5 and 0.5 cells on average per side).
void choose_tiles(Layout *L, int cus)
{
    if (cus < 1) cus = 1;
    double best = -1.0;
    for (int tx = L->ftile; tx >= mpmc::kFusedMinTile; tx -= 2)
        for (int ty = L->ftile; ty >= mpmc::kFusedMinTile; ty -= 2) {
            long long tiles = 0;
            for (const Rep &R : L->reps)
                tiles += (long long)((R.g.mx + tx - 1) / tx) * ((R.g.my + ty - 1) / ty);
            double work = 0.0;
            for (int p = 1; p <= 4; ++p)
                work += (tx + 2.0 * (4 - p) + 0.5) * (ty + 2.0 * (4 - p) + 0.5);
            const double cost = (double)((tiles + cus - 1) / cus) * work + 1e-9 * (double)tiles * work;
            if (best < 0.0 || cost < best) {
                best = cost;
                L->ftx = tx;
                L->fty = ty;
            }
        }
    L->ftiles = 0;
    for (Rep &R : L->reps) {
        R.tiles_x = (R.g.mx + L->ftx - 1) / L->ftx;
        R.tiles_y = (R.g.my + L->fty - 1) / L->fty;
        R.tb = L->ftiles;
        L->ftiles += (long long)R.tiles_x * R.tiles_y;
    }
}

mpmc_status plan(const mpmc_params *p, int n, Layout *L)
{
    if (!p || n < 1) return fail(MPMC_EINVAL, "need at least one replica");
    if (n > kMaxReplicas) return fail(MPMC_EINVAL, "too many replicas");
    L->geo.resize((size_t)n);
    L->reps.resize((size_t)n);
    L->N = L->cells = L->active = 0;
    L->cap = 0;
    for (int r = 0; r < n; ++r) {
        mpmc_status s = derive_geometry(&p[r], &L->geo[(size_t)r]);
        if (s) return s;
        s = check_params(&p[r], L->geo[(size_t)r]);
        if (s) return s;
        if ((p[r].flags ^ p[0].flags) & ~kChainFlags)
            return fail(MPMC_EINVAL, "replicas must share the buffer flags (ACC, TAG, ACCEPT_LOG)");
        const mpmc_geometry &g = L->geo[(size_t)r];
        Rep &R = L->reps[(size_t)r];
        std::memset(&R, 0, sizeof R);
        R.g.mx = g.cells_x;
        R.g.my = g.cells_y;
        R.g.C = g.cells_x * g.cells_y;
        R.g.cap = g.capacity;
        R.g.wx = g.w_x;
        R.g.wy = g.w_y;
        R.g.N = g.n_particles;
        R.cb = L->cells;
        // at least one padding cell: the end offset of the last real cell is
        // then always the replica's own entry (see the placeholder below)
        R.cpad = round_up((long long)R.g.C + 1, mpmc::kRebinTile);
        R.pb = L->N;
        R.ab = L->active;
        R.apad = round_up((long long)(g.cells_x / 2) * (g.cells_y / 2), mpmc::kActiveChunk);
        R.n_moves = p[r].n_moves;
        R.key0 = p[r].seed;
        R.key1 = p[r].replica;
        R.delta0 = p[r].delta;
        R.disk = (p[r].flags & MPMC_FLAG_DISK) ? 1 : 0;
        R.ablate = ((p[r].flags & MPMC_FLAG_NO_PARTICLE_SHUFFLE) ? mpmc::kAblateParticleShuffle : 0) |
                   ((p[r].flags & MPMC_FLAG_NO_SET_SHUFFLE) ? mpmc::kAblateSetShuffle : 0) |
                   ((p[r].flags & MPMC_FLAG_LEAVE) ? mpmc::kAblateLeave : 0) |
                   ((p[r].flags & MPMC_FLAG_LEAVE_ONCE) ? mpmc::kAblateLeaveOnce : 0);
        // tiles of the fused sweep at the smallest shape (an upper bound for
        // the tile table; the shape is chosen when the handle is built)
        L->ftile = mpmc::fused_tile((p[0].flags & MPMC_FLAG_ACC) != 0, (p[0].flags & MPMC_FLAG_TAG) != 0);
        const int mt = mpmc::kFusedMinTile;
        L->ftiles_max += (long long)((g.cells_x + mt - 1) / mt) * ((g.cells_y + mt - 1) / mt);
        L->cells += R.cpad;
        L->N += R.g.N;
        L->active += R.apad;
        L->cap = std::max(L->cap, R.g.cap);
    }
    if (L->ftiles_max > 0x7FFFFF00LL) return fail(MPMC_EGEOM, "too many cells");
    choose_tiles(L, 256);   // a default shape; the handle re-chooses for its device
    if (L->N > 0xFFFFFF00LL) return fail(MPMC_EGEOM, "too many disks (32-bit offsets)");
    if (L->cells > 0x7FFFFF00LL) return fail(MPMC_EGEOM, "too many cells");
    return MPMC_OK;
}

size_t work_bytes(const Layout &L)
{
    return align256((size_t)mpmc::count_stride(L.active) * 2 * 8) +
           align256((size_t)mpmc::kMsdBlocksMax * sizeof(double)) +
           (size_t)L.active * mpmc::ovf_per_slot(L.cap) * 8 + 256;
}

// Control buffer: Ctl[R], Rep[R], replica of each active chunk, replica of
// each rebin tile.
struct CtlLayout {
    size_t reps, arep, crep, trep, total;
};

CtlLayout ctl_layout(const Layout &L)
{
    const size_t R = L.reps.size();
    CtlLayout c;
    c.reps = align256(R * sizeof(Ctl));
    c.arep = c.reps + align256(R * sizeof(Rep));
    c.crep = c.arep + align256((size_t)(L.active / mpmc::kActiveChunk) * 2);
    c.trep = c.crep + align256((size_t)(L.cells / mpmc::kRebinTile) * 2);
    c.total = c.trep + align256((size_t)L.ftiles_max * 2);
    return c;
}

mpmc_status sizes_of(const mpmc_params *p, int n, mpmc_buffer_sizes *out)
{
    if (!out) return fail(MPMC_EINVAL, "null argument");
    Layout L;
    const mpmc_status s = plan(p, n, &L);
    if (s) return s;
    const size_t slots = (size_t)L.cells * (size_t)L.cap;   // L.cap slots per cell
    out->pos = align256(8 * slots);
    out->count = align256(4 * (size_t)L.cells);
    out->acc = (p[0].flags & MPMC_FLAG_ACC) ? align256(8 * slots) : 0;
    out->tag = (p[0].flags & MPMC_FLAG_TAG) ? align256(4 * slots) : 0;
    out->work = work_bytes(L);
    out->ctl = ctl_layout(L).total;
    out->accept_log = (p[0].flags & MPMC_FLAG_ACCEPT_LOG) ? align256(4 * (size_t)L.cells) : 0;
    return MPMC_OK;
}

}  // namespace

struct mpmc_system {
    std::vector<mpmc_params> p;
    Layout L;
    mpmc::Tables t;
    hipStream_t st;
    float2 *pos[2];     // slots: t.cap per cell
    uint32_t *count[2]; // disks per cell
    float2 *acc[2];
    uint32_t *tag[2];
    mpmc::Work work;
    int cur;
    int block;                    // sub-sweep workgroup size
    int lanes;                    // sub-sweep lanes per active cell
    bool fused;                   // whole sweeps in one tiled launch where supported
    uint32_t *alog;               // per-cell accept bits, or null
    std::vector<uint32_t> key0;   // current key word 0 of each replica
    std::vector<char> loaded;     // replica holds a valid, overlap-free state
    bool ready;                   // every replica is loaded
    hipGraphExec_t graph[2];      // kGraphSweeps sweeps from ping-pong half 0 / 1
    hipGraphExec_t tail[2];       // tail_n[p] (< kGraphSweeps) sweeps from half p
    int tail_n[2];
    std::vector<Ctl> ctl_host;
    int R() const { return (int)p.size(); }
};

namespace {

void drop_graphs(mpmc_system *h)
{
    for (int i = 0; i < 2; ++i) {
        if (h->graph[i]) {
            (void)hipGraphExecDestroy(h->graph[i]);
            h->graph[i] = nullptr;
        }
        if (h->tail[i]) {
            (void)hipGraphExecDestroy(h->tail[i]);
            h->tail[i] = nullptr;
        }
        h->tail_n[i] = 0;
    }
}

// Fold the counter partials, copy every control block to the host, wait,
// and report a device error word.
mpmc_status read_ctl(mpmc_system *h)
{
    MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
    MPMC_HIP(hipMemcpyAsync(h->ctl_host.data(), h->t.ctls, sizeof(Ctl) * (size_t)h->R(),
                            hipMemcpyDeviceToHost, h->st));
    MPMC_HIP(hipStreamSynchronize(h->st));
    for (int r = 0; r < h->R(); ++r) {
        const unsigned e = h->ctl_host[(size_t)r].errword;
        if (e) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "device invariant violated in replica %d (error word 0x%x)%s",
                          r, e, (e & mpmc::kErrCapacity) ? ": cell above capacity" : "");
            return fail(MPMC_EDEVICE, buf);
        }
    }
    return MPMC_OK;
}

mpmc_status enqueue_subsweep(mpmc_system *h, int set)
{
    MPMC_HIP(mpmc::launch_subsweep(h->t, h->cur, h->pos[h->cur], h->count[h->cur], h->acc[h->cur],
                                   h->tag[h->cur], h->alog, h->work, set, h->block, h->lanes,
                                   h->st));
    return MPMC_OK;
}

mpmc_status enqueue_rebin(mpmc_system *h, int f, float d, int advance)
{
    const int o = h->cur ^ 1;
    MPMC_HIP(mpmc::launch_rebin(h->t, h->cur, h->pos[h->cur], h->count[h->cur], h->acc[h->cur],
                                h->tag[h->cur], h->pos[o], h->count[o], h->acc[o], h->tag[o],
                                h->work, f, d, advance, h->st));
    h->cur = o;
    return MPMC_OK;
}

bool use_fused(const mpmc_system *h) { return h->fused && mpmc::sweep_fused_supported(h->t); }

mpmc_status enqueue_sweep(mpmc_system *h)
{
    if (use_fused(h)) {
        const int c = h->cur, o = c ^ 1;
        MPMC_HIP(mpmc::launch_sweep_fused(h->t, c, h->pos[c], h->count[c], h->acc[c], h->tag[c],
                                          h->pos[o], h->count[o], h->acc[o], h->tag[o], h->alog,
                                          h->work, h->st));
        h->cur = o;
        return MPMC_OK;
    }
    for (int slot = 0; slot < 4; ++slot) {
        const mpmc_status s = enqueue_subsweep(h, -1 - slot);
        if (s) return s;
    }
    return enqueue_rebin(h, -1, 0.0f, 1);
}

// Capture n sweeps starting from the current ping-pong half into *ex (the
// stream is only recorded, nothing runs).
mpmc_status capture_sweeps(mpmc_system *h, int n, hipGraphExec_t *ex)
{
    const int cur0 = h->cur;
    hipGraph_t graph = nullptr;
    MPMC_HIP(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
    mpmc_status s = MPMC_OK;
    for (int k = 0; k < n && s == MPMC_OK; ++k) s = enqueue_sweep(h);
    const hipError_t e = hipStreamEndCapture(h->st, &graph);
    h->cur = cur0;
    if (s) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(MPMC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        *ex = nullptr;
        return fail(MPMC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    return MPMC_OK;
}

// Make sure the graphs that n sweeps from the current half launch exist:
// the kGraphSweeps graph of this half (an even count, so every full graph
// starts on the same half) and the graph of the n mod kGraphSweeps rest.
mpmc_status prepare_sweeps(mpmc_system *h, int64_t n)
{
    if (!h->st) return MPMC_OK;   // the null stream cannot be captured: eager launches
    const int p = h->cur;
    if (n >= kGraphSweeps && !h->graph[p]) {
        const mpmc_status s = capture_sweeps(h, kGraphSweeps, &h->graph[p]);
        if (s) return s;
    }
    const int rest = (int)(n % kGraphSweeps);
    if (rest > 0 && (!h->tail[p] || h->tail_n[p] != rest)) {
        if (h->tail[p]) {
            (void)hipGraphExecDestroy(h->tail[p]);
            h->tail[p] = nullptr;
            h->tail_n[p] = 0;
        }
        const mpmc_status s = capture_sweeps(h, rest, &h->tail[p]);
        if (s) return s;
        h->tail_n[p] = rest;
    }
    return MPMC_OK;
}

// n sweeps as graph launches only (eager launches on the null stream).
mpmc_status run_sweeps(mpmc_system *h, int64_t n)
{
    if (h->st) {
        const mpmc_status s = prepare_sweeps(h, n);
        if (s) return s;
        const int p = h->cur;
        for (int64_t k = 0; k < n / kGraphSweeps; ++k) MPMC_HIP(hipGraphLaunch(h->graph[p], h->st));
        const int rest = (int)(n % kGraphSweeps);
        if (rest > 0) {
            MPMC_HIP(hipGraphLaunch(h->tail[p], h->st));
            h->cur = p ^ (rest & 1);
        }
        return MPMC_OK;
    }
    for (; n > 0; --n) {
        const mpmc_status s = enqueue_sweep(h);
        if (s) return s;
    }
    return MPMC_OK;
}

// A replica's state in its own numbering: start[0] = 0, start[C] = N_r.
mpmc_status validate_host_state(const Rep &R, const float *xy, const uint32_t *start)
{
    const int C = R.g.C;
    if (start[0] != 0) return fail(MPMC_ESTATE, "start[0] != 0");
    for (int c = 0; c < C; ++c) {
        if (start[c + 1] < start[c]) return fail(MPMC_ESTATE, "offsets decrease");
        if (start[c + 1] - start[c] > (uint32_t)R.g.cap) return fail(MPMC_ESTATE, "cell above capacity");
    }
    if ((long long)start[C] != R.g.N) return fail(MPMC_ESTATE, "particle count differs from the buffers' N");
    for (long long k = 0; k < R.g.N; ++k) {
        const float x = xy[2 * k], y = xy[2 * k + 1];
        if (!(x > 0.0f && x <= R.g.wx && y > 0.0f && y <= R.g.wy))
            return fail(MPMC_ESTATE, "local coordinate outside (0, w]");
    }
    return MPMC_OK;
}

// A replica's compact lists (xy, start, tags in its own numbering) laid out
// in its slots: counts for its cpad cells (padding cells empty) and S slots
// per cell; unused slots hold zeros.
struct SlotState {
    std::vector<uint32_t> count;   // [cpad]
    std::vector<float> xy;         // [cpad * S * 2]
    std::vector<uint32_t> tag;     // [cpad * S]
};

void to_slots(const Rep &R, int S, const float *xy, const uint32_t *start, const uint32_t *tags,
              SlotState &o)
{
    const size_t cells = (size_t)R.cpad;
    o.count.assign(cells, 0u);
    o.xy.assign(cells * (size_t)S * 2, 0.0f);
    o.tag.assign(cells * (size_t)S, 0u);
    for (int c = 0; c < R.g.C; ++c) {
        const uint32_t b = start[c], n = start[c + 1] - start[c];
        o.count[(size_t)c] = n;
        for (uint32_t i = 0; i < n; ++i) {
            const size_t k = (size_t)c * S + i;
            o.xy[2 * k] = xy[2 * (size_t)(b + i)];
            o.xy[2 * k + 1] = xy[2 * (size_t)(b + i) + 1];
            o.tag[k] = tags ? tags[b + i] : b + i;
        }
    }
}

// Initial condition of a lattice replica (Sec. 4): site (i, j) at
// x = (i + 1/4 + (j odd)/2) a, y = (j + 1/2) h in FP64; cell ceil(x/w) - 1;
// local (float)(x - c w); cells list their disks in ascending lattice index.
mpmc_status build_lattice(const mpmc_params &p, const Rep &R, std::vector<float> &xy,
                          std::vector<uint32_t> &start, std::vector<uint32_t> &tags)
{
    const int nx = p.lattice_nx, ny = p.lattice_ny;
    const long long N = R.g.N;
    const int C = R.g.C;
    const Lattice Lt = lattice_of(nx, ny, p.phi);
    start.assign((size_t)C + 1, 0);
    xy.assign(2 * (size_t)N, 0.0f);
    tags.assign((size_t)N, 0);
    std::vector<int> cell_of((size_t)N);
    std::vector<float> lx((size_t)N), ly((size_t)N);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            const double x = ((double)i + 0.25 + 0.5 * (double)(j & 1)) * Lt.a;
            const double y = ((double)j + 0.5) * Lt.h;
            const int cx = (int)std::ceil(x / (double)R.g.wx) - 1;
            const int cy = (int)std::ceil(y / (double)R.g.wy) - 1;
            if (cx < 0 || cx >= R.g.mx || cy < 0 || cy >= R.g.my)
                return fail(MPMC_EGEOM, "lattice site outside the cell grid");
            lx[k] = (float)(x - (double)cx * (double)R.g.wx);
            ly[k] = (float)(y - (double)cy * (double)R.g.wy);
            cell_of[k] = cy * R.g.mx + cx;
            start[(size_t)cell_of[k] + 1] += 1;
        }
    for (int c = 0; c < C; ++c) start[(size_t)c + 1] += start[(size_t)c];
    std::vector<uint32_t> fill(start.begin(), start.end() - 1);
    for (long long k = 0; k < N; ++k) {
        const uint32_t o = fill[(size_t)cell_of[(size_t)k]]++;
        xy[2 * (size_t)o] = lx[(size_t)k];
        xy[2 * (size_t)o + 1] = ly[(size_t)k];
        tags[o] = (uint32_t)k;
    }
    return validate_host_state(R, xy.data(), start.data());
}

// Copy a replica's counts (and, if asked, one float2 slot array) to the host;
// the caller synchronises (read_ctl) before using them.
mpmc_status read_slots(mpmc_system *h, const Rep &R, const float2 *dev, std::vector<float2> *out,
                       std::vector<uint32_t> &cnt)
{
    const size_t S = (size_t)h->t.cap, n = (size_t)R.g.C * S;
    cnt.resize(std::max<size_t>((size_t)R.g.C, 1));
    if (R.g.C > 0)
        MPMC_HIP(hipMemcpyAsync(cnt.data(), h->count[h->cur] + R.cb, sizeof(uint32_t) * (size_t)R.g.C,
                                hipMemcpyDeviceToHost, h->st));
    if (out && dev) {
        out->resize(std::max<size_t>(n, 1));
        if (n) MPMC_HIP(hipMemcpyAsync(out->data(), dev + (size_t)R.cb * S, sizeof(float2) * n,
                                       hipMemcpyDeviceToHost, h->st));
    }
    return MPMC_OK;
}

// Slots -> compact lists in the replica's own numbering: xy (if both given)
// and start[C + 1] (if given).  Fails if the counts do not add up to N.
mpmc_status compact_lists(const Rep &R, int S, const std::vector<uint32_t> &cnt, const float2 *slots,
                          float2 *xy, uint32_t *start)
{
    uint64_t total = 0;
    for (int c = 0; c < R.g.C; ++c) {
        if (cnt[(size_t)c] > (uint32_t)R.g.cap) return fail(MPMC_EDEVICE, "cell above capacity");
        total += cnt[(size_t)c];
    }
    if ((long long)total != R.g.N) return fail(MPMC_EDEVICE, "cell counts do not add up to N");
    uint32_t k = 0;
    for (int c = 0; c < R.g.C; ++c) {
        if (start) start[c] = k;
        for (uint32_t i = 0; i < cnt[(size_t)c]; ++i, ++k)
            if (slots && xy) xy[k] = slots[(size_t)c * S + i];
    }
    if (start) start[R.g.C] = k;
    return MPMC_OK;
}

// Overlap check of the loaded replicas in the kernels' metric; marks them
// loaded when clean.
mpmc_status check_loaded(mpmc_system *h, const std::vector<int> &which)
{
    MPMC_HIP(mpmc::launch_count_overlaps(h->t, h->pos[h->cur], h->count[h->cur], h->st));
    mpmc_status s = read_ctl(h);
    if (s) return s;
    for (int r : which)
        if (h->ctl_host[(size_t)r].overlaps != 0) {
            char buf[96];
            std::snprintf(buf, sizeof buf, "state of replica %d contains overlapping disks", r);
            return fail(MPMC_EOVERLAP, buf);
        }
    for (int r : which) h->loaded[(size_t)r] = 1;
    h->ready = std::all_of(h->loaded.begin(), h->loaded.end(), [](char c) { return c != 0; });
    return MPMC_OK;
}

// Load replica r's state into the current half (its cells and slots only).
mpmc_status upload_replica(mpmc_system *h, int r, const float *xy, const uint32_t *start,
                           uint64_t sweep, const uint32_t *tags)
{
    const Rep &R = h->L.reps[(size_t)r];
    const int S = h->t.cap;
    const size_t slots = (size_t)R.cpad * (size_t)S, s0 = (size_t)R.cb * (size_t)S;
    h->loaded[(size_t)r] = 0;
    h->ready = false;
    SlotState o;
    to_slots(R, S, xy, start, tags, o);
    const int c = h->cur;
    MPMC_HIP(hipMemcpyAsync(h->pos[c] + s0, o.xy.data(), sizeof(float2) * slots, hipMemcpyHostToDevice, h->st));
    MPMC_HIP(hipMemcpyAsync(h->count[c] + R.cb, o.count.data(), sizeof(uint32_t) * (size_t)R.cpad,
                            hipMemcpyHostToDevice, h->st));
    if (h->tag[c])
        MPMC_HIP(hipMemcpyAsync(h->tag[c] + s0, o.tag.data(), sizeof(uint32_t) * slots, hipMemcpyHostToDevice, h->st));
    if (h->acc[c]) MPMC_HIP(mpmc::launch_fill_u32((uint32_t *)(h->acc[c] + s0), 0u, 2 * (long long)slots, h->st));
    // counters of the other replicas are kept: fold them before the reset
    MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
    MPMC_HIP(mpmc::launch_ctl_reset(h->t, r, sweep, h->st));
    h->key0[(size_t)r] = R.key0;
    MPMC_HIP(hipStreamSynchronize(h->st));   // host arrays go out of scope
    return check_loaded(h, {r});
}

// Build a handle: copy the tables to the device, lay out the initial states
// (lattices where given, empty placeholders for the rest) and check them.
mpmc_status create(const mpmc_params *p, int n, const mpmc_buffers *b, void *stream,
                   mpmc_handle *out)
{
    if (!b || !out) return fail(MPMC_EINVAL, "null argument");
    *out = nullptr;
    Layout L;
    mpmc_status s = plan(p, n, &L);
    if (s) return s;
    const uint32_t flags = p[0].flags;
    for (int i = 0; i < 2; ++i) {
        if (!b->pos[i] || !b->count[i]) return fail(MPMC_EINVAL, "pos/count buffers missing");
        if ((flags & MPMC_FLAG_ACC) && !b->acc[i]) return fail(MPMC_EINVAL, "acc buffers missing");
        if ((flags & MPMC_FLAG_TAG) && !b->tag[i]) return fail(MPMC_EINVAL, "tag buffers missing");
    }
    if (!b->work || !b->ctl) return fail(MPMC_EINVAL, "work/ctl buffers missing");
    if ((flags & MPMC_FLAG_ACCEPT_LOG) && !b->accept_log)
        return fail(MPMC_EINVAL, "accept_log buffer missing");
    // host-side states first, so that geometry errors allocate nothing
    const int S = L.cap;
    std::vector<uint32_t> count_g((size_t)L.cells, 0u);
    std::vector<float> xy_g((size_t)L.cells * (size_t)S * 2, 0.0f);
    std::vector<uint32_t> tag_g((size_t)L.cells * (size_t)S, 0u);
    std::vector<int> lattice;
    for (int r = 0; r < n; ++r) {
        const Rep &R = L.reps[(size_t)r];
        if (p[r].lattice_nx > 0) {
            std::vector<float> xy;
            std::vector<uint32_t> st, tg;
            s = build_lattice(p[r], R, xy, st, tg);
            if (s) return s;
            SlotState o;
            to_slots(R, S, xy.data(), st.data(), tg.data(), o);
            std::copy(o.count.begin(), o.count.end(), count_g.begin() + R.cb);
            std::copy(o.xy.begin(), o.xy.end(), xy_g.begin() + 2 * (size_t)R.cb * S);
            std::copy(o.tag.begin(), o.tag.end(), tag_g.begin() + (size_t)R.cb * S);
            lattice.push_back(r);
        } else if (R.g.N == 0) {
            lattice.push_back(r);   // empty grid: already valid
        }
        // (other replicas: every cell empty until set_state)
    }

    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            choose_tiles(&L, cus);
    }
    mpmc_system *h = new mpmc_system();
    h->p.assign(p, p + n);
    h->L = L;
    h->st = (hipStream_t)stream;
    for (int i = 0; i < 2; ++i) {
        h->pos[i] = (float2 *)b->pos[i];
        h->count[i] = (uint32_t *)b->count[i];
        h->acc[i] = (flags & MPMC_FLAG_ACC) ? (float2 *)b->acc[i] : nullptr;
        h->tag[i] = (flags & MPMC_FLAG_TAG) ? (uint32_t *)b->tag[i] : nullptr;
    }
    {
        char *w = (char *)b->work;
        h->work.cnt = (unsigned long long *)w;
        h->work.cnt_stride = (int)mpmc::count_stride(L.active);
        w += align256((size_t)mpmc::count_stride(L.active) * 2 * 8);
        h->work.f64 = (double *)w;
        w += align256((size_t)mpmc::kMsdBlocksMax * sizeof(double));
        h->work.ovf = (float2 *)w;
    }
    const CtlLayout cl = ctl_layout(L);
    char *cb = (char *)b->ctl;
    h->t.ctls = (Ctl *)cb;
    h->t.reps = (const Rep *)(cb + cl.reps);
    h->t.arep = (const uint16_t *)(cb + cl.arep);
    h->t.crep = (const uint16_t *)(cb + cl.crep);
    h->t.trep = (const uint16_t *)(cb + cl.trep);
    h->t.ftiles = L.ftiles;
    h->t.ftile = L.ftile;
    h->t.ftx = L.ftx;
    h->t.fty = L.fty;
    h->t.rep0 = L.reps[0];
    h->t.R = n;
    h->t.cap = L.cap;
    {
        int ndisk = 0, noshuf = 0, nleave = 0;
        for (const Rep &R : L.reps) {
            ndisk += R.disk;
            noshuf += (R.ablate & mpmc::kAblateParticleShuffle) ? 1 : 0;
            nleave += (R.ablate & (mpmc::kAblateLeave | mpmc::kAblateLeaveOnce)) ? 1 : 0;
        }
        h->t.prop = (noshuf > 0 || nleave > 0) ? 2 : (ndisk == 0 ? 0 : (ndisk == n ? 1 : 2));
        h->t.leave = nleave > 0 ? 1 : 0;
    }
    h->t.cells = L.cells;
    h->t.active = L.active;
    h->t.N = L.N;
    h->alog = (flags & MPMC_FLAG_ACCEPT_LOG) ? (uint32_t *)b->accept_log : nullptr;
    h->cur = 0;
    h->block = 256;
    h->lanes = 1;
    h->fused = true;
    h->key0.resize((size_t)n);
    for (int r = 0; r < n; ++r) h->key0[(size_t)r] = p[r].seed;
    h->loaded.assign((size_t)n, 0);
    h->ready = false;
    h->graph[0] = h->graph[1] = nullptr;
    h->tail[0] = h->tail[1] = nullptr;
    h->tail_n[0] = h->tail_n[1] = 0;
    h->ctl_host.resize((size_t)n);

    std::vector<uint16_t> arep((size_t)(L.active / mpmc::kActiveChunk));
    std::vector<uint16_t> crep((size_t)(L.cells / mpmc::kRebinTile));
    std::vector<uint16_t> trep((size_t)L.ftiles);
    for (int r = 0; r < n; ++r) {
        const Rep &R = L.reps[(size_t)r];
        for (long long i = R.tb; i < R.tb + (long long)R.tiles_x * R.tiles_y; ++i)
            trep[(size_t)i] = (uint16_t)r;
        for (long long i = R.ab / mpmc::kActiveChunk; i < (R.ab + R.apad) / mpmc::kActiveChunk; ++i)
            arep[(size_t)i] = (uint16_t)r;
        for (long long i = R.cb / mpmc::kRebinTile; i < (R.cb + R.cpad) / mpmc::kRebinTile; ++i)
            crep[(size_t)i] = (uint16_t)r;
    }
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->st) : hipSuccess;
    };
    hipError_t e = up(cb + cl.reps, L.reps.data(), sizeof(Rep) * (size_t)n);
    if (e == hipSuccess) e = up(cb + cl.arep, arep.data(), arep.size() * 2);
    if (e == hipSuccess) e = up(cb + cl.crep, crep.data(), crep.size() * 2);
    if (e == hipSuccess) e = up(cb + cl.trep, trep.data(), trep.size() * 2);
    const long long slots = L.cells * (long long)S;
    if (e == hipSuccess) e = up(h->pos[0], xy_g.data(), sizeof(float2) * (size_t)slots);
    if (e == hipSuccess) e = up(h->count[0], count_g.data(), sizeof(uint32_t) * count_g.size());
    // the other half: counts of padding cells are read by nothing but kept 0
    if (e == hipSuccess) e = mpmc::launch_fill_u32(h->count[1], 0u, L.cells, h->st);
    if (e == hipSuccess && h->tag[0]) e = up(h->tag[0], tag_g.data(), sizeof(uint32_t) * (size_t)slots);
    if (e == hipSuccess && h->acc[0]) e = mpmc::launch_fill_u32((uint32_t *)h->acc[0], 0u, 2 * slots, h->st);

    if (e == hipSuccess)
        e = mpmc::launch_fill_u32((uint32_t *)h->work.cnt, 0u, 4LL * h->work.cnt_stride, h->st);
    if (e == hipSuccess && h->alog) e = mpmc::launch_fill_u32(h->alog, 0u, L.cells, h->st);
    if (e == hipSuccess) e = mpmc::launch_ctl_reset(h->t, -1, 0, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
        delete h;
        return fail(MPMC_EHIP, std::string("init upload: ") + hipGetErrorString(e));
    }
    s = check_loaded(h, lattice);
    if (s) {
        delete h;
        return s;
    }
    *out = h;
    return MPMC_OK;
}

#define MPMC_NEED_STATE(h)                                                                   \
    do {                                                                                     \
        if (!(h)) return fail(MPMC_EINVAL, "null handle");                                   \
        if (!(h)->ready) return fail(MPMC_ESTATE, "no valid state loaded (mpmc_set_state)"); \
    } while (0)

#define MPMC_NEED_REPLICA(h, r)                                                              \
    do {                                                                                     \
        if (!(h)) return fail(MPMC_EINVAL, "null handle");                                   \
        if ((r) < 0 || (r) >= (h)->R()) return fail(MPMC_EINVAL, "replica out of range");    \
    } while (0)

#define MPMC_NEED_LOADED(h, r)                                                               \
    do {                                                                                     \
        MPMC_NEED_REPLICA(h, r);                                                             \
        if (!(h)->loaded[(size_t)(r)])                                                       \
            return fail(MPMC_ESTATE, "no valid state loaded (mpmc_set_state)");              \
    } while (0)

#define MPMC_NEED_SINGLE(h)                                                                  \
    do {                                                                                     \
        if (!(h)) return fail(MPMC_EINVAL, "null handle");                                   \
        if ((h)->R() != 1) return fail(MPMC_EINVAL, "batched handle: use mpmc_replica_*");   \
    } while (0)

mpmc_status check_delta(const mpmc_system *h, int r, float delta)
{
    const Geom &g = h->L.reps[(size_t)r].g;
    if (!(delta > 0.0f) || delta > 0.5f * std::min(g.wx, g.wy))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    return MPMC_OK;
}

}  // namespace

namespace mpmc {
// The calling thread's last failure message, shared with the sphere calls.
void set_last_error(const char *msg) { g_last_error = msg; }
}  // namespace mpmc

extern "C" {

const char *mpmc_last_error(void) { return g_last_error.c_str(); }

mpmc_status mpmc_geometry_of(const mpmc_params *p, mpmc_geometry *out)
{
    return derive_geometry(p, out);
}

mpmc_status mpmc_required_bytes(const mpmc_params *p, mpmc_buffer_sizes *out)
{
    if (!p) return fail(MPMC_EINVAL, "null argument");
    return sizes_of(p, 1, out);
}

mpmc_status mpmc_batch_required_bytes(const mpmc_params *per_replica, int32_t n_replicas,
                                      mpmc_buffer_sizes *out)
{
    return sizes_of(per_replica, n_replicas, out);
}

mpmc_status mpmc_init_system(const mpmc_params *p, const mpmc_buffers *b, void *stream,
                             mpmc_handle *out)
{
    if (!p) return fail(MPMC_EINVAL, "null argument");
    return create(p, 1, b, stream, out);
}

mpmc_status mpmc_batch_init(const mpmc_params *per_replica, int32_t n_replicas,
                            const mpmc_buffers *b, void *stream, mpmc_handle *out)
{
    return create(per_replica, n_replicas, b, stream, out);
}

mpmc_status mpmc_num_replicas(mpmc_handle h, int32_t *n)
{
    if (!h || !n) return fail(MPMC_EINVAL, "null argument");
    *n = h->R();
    return MPMC_OK;
}

mpmc_status mpmc_replica_geometry(mpmc_handle h, int32_t r, mpmc_geometry *out)
{
    MPMC_NEED_REPLICA(h, r);
    if (!out) return fail(MPMC_EINVAL, "null argument");
    *out = h->L.geo[(size_t)r];
    return MPMC_OK;
}

mpmc_status mpmc_sweep(mpmc_handle h, int64_t n_sweeps, uint32_t seed)
{
    if (!h || n_sweeps < 0) return fail(MPMC_EINVAL, "bad handle or sweep count");
    MPMC_NEED_STATE(h);
    if (std::any_of(h->key0.begin(), h->key0.end(), [&](uint32_t k) { return k != seed; })) {
        MPMC_HIP(mpmc::launch_ctl_set_key0(h->t, seed, h->st));
        std::fill(h->key0.begin(), h->key0.end(), seed);
    }
    return run_sweeps(h, n_sweeps);
}

mpmc_status mpmc_prepare_sweeps(mpmc_handle h, int64_t n_sweeps)
{
    if (!h || n_sweeps < 0) return fail(MPMC_EINVAL, "bad handle or sweep count");
    MPMC_NEED_STATE(h);
    return prepare_sweeps(h, n_sweeps);
}

mpmc_status mpmc_subsweep(mpmc_handle h, int32_t set)
{
    if (!h || set < 0 || set > 3) return fail(MPMC_EINVAL, "set must be 0..3");
    MPMC_NEED_STATE(h);
    return enqueue_subsweep(h, set);
}

mpmc_status mpmc_shift_and_rebin(mpmc_handle h, int32_t f, float d)
{
    if (!h || f < -1 || f > 3) return fail(MPMC_EINVAL, "f must be -1..3");
    if (f >= 0)
        for (const Rep &R : h->L.reps) {
            const float w = f < 2 ? R.g.wx : R.g.wy;
            if (!(d >= 0.0f && d <= 0.5f * w)) return fail(MPMC_EINVAL, "d must lie in [0, w/2]");
        }
    MPMC_NEED_STATE(h);
    if (f >= 0) return enqueue_rebin(h, f, d, 0);
    return enqueue_rebin(h, -1, 0.0f, 1);
}

mpmc_status mpmc_pair_histogram(mpmc_handle h, int32_t reset)
{
    MPMC_NEED_STATE(h);
    const double rmax = 1.0 + MPMC_HIST_BINS * 1e-4;
    for (const Rep &R : h->L.reps) {
        const int Rx = (double)R.g.wx >= rmax ? 1 : 2, Ry = (double)R.g.wy >= rmax ? 1 : 2;
        if (R.g.mx < 2 * Rx + 2 || R.g.my < 2 * Ry + 2)
            return fail(MPMC_EGEOM, "grid too small for the histogram's reach");
    }
    MPMC_HIP(mpmc::launch_pair_histogram(h->t, h->pos[h->cur], h->count[h->cur], reset, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_replica_pressure_from_contact(mpmc_handle h, int32_t r, double *p_star,
                                               double *g_contact, uint64_t *hist,
                                               uint64_t *n_samples)
{
    MPMC_NEED_LOADED(h, r);
    mpmc_status s = read_ctl(h);
    if (s) return s;
    if (h->ctl_host[(size_t)r].hist_samples == 0) {
        if (h->R() != 1) return fail(MPMC_ESTATE, "no histogram accumulated for this replica");
        s = mpmc_pair_histogram(h, 1);
        if (s) return s;
    }
    MPMC_HIP(mpmc::launch_pressure_fit(h->t, r, h->st));
    s = read_ctl(h);
    if (s) return s;
    const Ctl &c = h->ctl_host[(size_t)r];
    if (c.fit[3] != 1.0) return fail(MPMC_EDEVICE, "pressure fit failed");
    if (p_star) *p_star = c.fit[0];
    if (g_contact) *g_contact = c.fit[1];
    if (hist) std::memcpy(hist, c.hist, sizeof(c.hist));
    if (n_samples) *n_samples = c.hist_samples;
    return MPMC_OK;
}

mpmc_status mpmc_pressure_from_contact(mpmc_handle h, double *p_star, double *g_contact,
                                       uint64_t *hist, uint64_t *n_samples)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_pressure_from_contact(h, 0, p_star, g_contact, hist, n_samples);
}

mpmc_status mpmc_replica_get_state(mpmc_handle h, int32_t r, float *xy, uint32_t *start,
                                   uint64_t *sweep)
{
    MPMC_NEED_LOADED(h, r);
    const Rep &R = h->L.reps[(size_t)r];
    std::vector<uint32_t> cnt;
    std::vector<float2> slots;
    mpmc_status s = read_slots(h, R, h->pos[h->cur], xy ? &slots : nullptr, cnt);
    if (s) return s;
    s = read_ctl(h);
    if (s) return s;
    s = compact_lists(R, h->t.cap, cnt, xy ? slots.data() : nullptr, (float2 *)xy, start);
    if (s) return s;
    if (sweep) *sweep = h->ctl_host[(size_t)r].sweep_at[h->cur];
    return MPMC_OK;
}

mpmc_status mpmc_get_state(mpmc_handle h, float *xy, uint32_t *start, uint64_t *sweep)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_get_state(h, 0, xy, start, sweep);
}

mpmc_status mpmc_replica_set_state(mpmc_handle h, int32_t r, const float *xy,
                                   const uint32_t *start, uint64_t sweep, const uint32_t *tags)
{
    MPMC_NEED_REPLICA(h, r);
    const Rep &R = h->L.reps[(size_t)r];
    if (!start || (!xy && R.g.N > 0)) return fail(MPMC_EINVAL, "null argument");
    const mpmc_status s = validate_host_state(R, xy, start);
    if (s) return s;
    return upload_replica(h, r, xy, start, sweep, tags);
}

mpmc_status mpmc_set_state(mpmc_handle h, const float *xy, const uint32_t *start, uint64_t sweep,
                           const uint32_t *tags)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_set_state(h, 0, xy, start, sweep, tags);
}

mpmc_status mpmc_replica_get_aux(mpmc_handle h, int32_t r, float *acc, uint32_t *tags)
{
    MPMC_NEED_LOADED(h, r);
    const Rep &R = h->L.reps[(size_t)r];
    if (acc && !h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    if (tags && !h->tag[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_TAG");
    std::vector<uint32_t> cnt;
    std::vector<float2> as;
    mpmc_status s = read_slots(h, R, acc ? h->acc[h->cur] : nullptr, acc ? &as : nullptr, cnt);
    if (s) return s;
    std::vector<uint32_t> ts;
    if (tags) {
        const size_t S = (size_t)h->t.cap, n = (size_t)R.g.C * S;
        ts.resize(std::max<size_t>(n, 1));
        if (n) MPMC_HIP(hipMemcpyAsync(ts.data(), h->tag[h->cur] + (size_t)R.cb * S, sizeof(uint32_t) * n,
                                       hipMemcpyDeviceToHost, h->st));
    }
    s = read_ctl(h);
    if (s) return s;
    s = compact_lists(R, h->t.cap, cnt, acc ? as.data() : nullptr, (float2 *)acc, nullptr);
    if (s) return s;
    if (tags) {
        const int S = h->t.cap;
        size_t k = 0;
        for (int c = 0; c < R.g.C; ++c)
            for (uint32_t i = 0; i < cnt[(size_t)c]; ++i) tags[k++] = ts[(size_t)c * S + i];
    }
    return MPMC_OK;
}

mpmc_status mpmc_replica_set_acc(mpmc_handle h, int32_t r, const float *acc)
{
    MPMC_NEED_LOADED(h, r);
    if (!acc) return fail(MPMC_EINVAL, "null argument");
    if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    const Rep &R = h->L.reps[(size_t)r];
    std::vector<uint32_t> cnt;
    mpmc_status s = read_slots(h, R, nullptr, nullptr, cnt);
    if (s) return s;
    s = read_ctl(h);   // waits for the counts
    if (s) return s;
    const size_t S = (size_t)h->t.cap, n = (size_t)R.g.C * S;
    std::vector<float2> slots(std::max<size_t>(n, 1), make_float2(0.0f, 0.0f));
    size_t k = 0;
    for (int c = 0; c < R.g.C; ++c)
        for (uint32_t i = 0; i < cnt[(size_t)c]; ++i, ++k)
            slots[(size_t)c * S + i] = make_float2(acc[2 * k], acc[2 * k + 1]);
    if ((long long)k != R.g.N) return fail(MPMC_EDEVICE, "cell counts do not add up to N");
    if (n) MPMC_HIP(hipMemcpyAsync(h->acc[h->cur] + (size_t)R.cb * S, slots.data(), sizeof(float2) * n,
                                   hipMemcpyHostToDevice, h->st));
    MPMC_HIP(hipStreamSynchronize(h->st));   // the host array goes out of scope
    return MPMC_OK;
}

mpmc_status mpmc_set_acc(mpmc_handle h, const float *acc)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_set_acc(h, 0, acc);
}

mpmc_status mpmc_get_aux(mpmc_handle h, float *acc, uint32_t *tags)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_get_aux(h, 0, acc, tags);
}

mpmc_status mpmc_replica_get_accept_log(mpmc_handle h, int32_t r, uint32_t *bits)
{
    MPMC_NEED_LOADED(h, r);
    if (!bits) return fail(MPMC_EINVAL, "null argument");
    if (!h->alog) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACCEPT_LOG");
    const Rep &R = h->L.reps[(size_t)r];
    MPMC_HIP(hipMemcpyAsync(bits, h->alog + R.cb, sizeof(uint32_t) * (size_t)R.g.C,
                            hipMemcpyDeviceToHost, h->st));
    return read_ctl(h);
}

mpmc_status mpmc_get_accept_log(mpmc_handle h, uint32_t *bits)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_get_accept_log(h, 0, bits);
}

mpmc_status mpmc_reset_acc(mpmc_handle h)
{
    MPMC_NEED_STATE(h);
    if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    MPMC_HIP(mpmc::launch_fill_u32((uint32_t *)h->acc[h->cur], 0u, 2 * h->L.cells * (long long)h->t.cap,
                                   h->st));
    return MPMC_OK;
}

mpmc_status mpmc_replica_msd(mpmc_handle h, int32_t r, double *msd)
{
    MPMC_NEED_LOADED(h, r);
    if (!msd) return fail(MPMC_EINVAL, "null argument");
    if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    const Rep &R = h->L.reps[(size_t)r];
    MPMC_HIP(mpmc::launch_msd(h->t, r, R.g.N, h->acc[h->cur], h->count[h->cur], h->work, h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    *msd = h->ctl_host[(size_t)r].msd;
    return MPMC_OK;
}

mpmc_status mpmc_msd(mpmc_handle h, double *msd)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_msd(h, 0, msd);
}

mpmc_status mpmc_count_overlaps(mpmc_handle h, int64_t *pairs)
{
    MPMC_NEED_STATE(h);
    if (!pairs) return fail(MPMC_EINVAL, "null argument");
    MPMC_HIP(mpmc::launch_count_overlaps(h->t, h->pos[h->cur], h->count[h->cur], h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    int64_t total = 0;
    for (const Ctl &c : h->ctl_host) total += c.overlaps;
    *pairs = total;
    return MPMC_OK;
}

mpmc_status mpmc_replica_get_counters(mpmc_handle h, int32_t r, uint64_t *trials,
                                      uint64_t *accepts)
{
    MPMC_NEED_REPLICA(h, r);
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    if (trials) *trials = h->ctl_host[(size_t)r].trials;
    if (accepts) *accepts = h->ctl_host[(size_t)r].accepts;
    return MPMC_OK;
}

mpmc_status mpmc_get_counters(mpmc_handle h, uint64_t *trials, uint64_t *accepts)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    uint64_t t = 0, a = 0;
    for (const Ctl &c : h->ctl_host) {
        t += c.trials;
        a += c.accepts;
    }
    if (trials) *trials = t;
    if (accepts) *accepts = a;
    return MPMC_OK;
}

mpmc_status mpmc_replica_set_delta(mpmc_handle h, int32_t r, float delta)
{
    MPMC_NEED_REPLICA(h, r);
    const mpmc_status s = check_delta(h, r, delta);
    if (s) return s;
    MPMC_HIP(mpmc::launch_ctl_set_delta(h->t, r, delta, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_set_delta(mpmc_handle h, float delta)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    for (int r = 0; r < h->R(); ++r) {
        const mpmc_status s = check_delta(h, r, delta);
        if (s) return s;
    }
    MPMC_HIP(mpmc::launch_ctl_set_delta(h->t, -1, delta, h->st));
    return MPMC_OK;
}

// n_M lives in the replica table (and, for replica 0, in the kernel
// arguments captured by the sweep graphs): rewrite both, drop the graphs.
static mpmc_status set_n_moves(mpmc_system *h, int r0, int r1, int32_t n_moves)
{
    if (n_moves < 0 || n_moves > (1 << 20)) return fail(MPMC_EINVAL, "n_moves out of range");
    MPMC_HIP(hipStreamSynchronize(h->st));   // no launch in flight reads the table
    for (int r = r0; r < r1; ++r) {
        h->L.reps[(size_t)r].n_moves = n_moves;
        h->p[(size_t)r].n_moves = n_moves;
        MPMC_HIP(hipMemcpyAsync((Rep *)h->t.reps + r, &h->L.reps[(size_t)r], sizeof(Rep),
                                hipMemcpyHostToDevice, h->st));
    }
    h->t.rep0 = h->L.reps[0];
    drop_graphs(h);
    MPMC_HIP(hipStreamSynchronize(h->st));
    return MPMC_OK;
}

mpmc_status mpmc_set_n_moves(mpmc_handle h, int32_t n_moves)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    return set_n_moves(h, 0, h->R(), n_moves);
}

mpmc_status mpmc_replica_set_n_moves(mpmc_handle h, int32_t r, int32_t n_moves)
{
    MPMC_NEED_REPLICA(h, r);
    return set_n_moves(h, r, r + 1, n_moves);
}

mpmc_status mpmc_replica_get_delta(mpmc_handle h, int32_t r, float *delta)
{
    MPMC_NEED_REPLICA(h, r);
    if (!delta) return fail(MPMC_EINVAL, "null argument");
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    *delta = h->ctl_host[(size_t)r].delta;
    return MPMC_OK;
}

mpmc_status mpmc_get_delta(mpmc_handle h, float *delta)
{
    MPMC_NEED_SINGLE(h);
    return mpmc_replica_get_delta(h, 0, delta);
}

mpmc_status mpmc_tune(mpmc_handle h, int32_t window_sweeps, int32_t n_windows)
{
    if (!h || window_sweeps < 1 || n_windows < 0) return fail(MPMC_EINVAL, "bad tuner arguments");
    MPMC_NEED_STATE(h);
    MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
    MPMC_HIP(mpmc::launch_tune(h->t, 0, h->st));   // open the first window
    for (int w = 0; w < n_windows; ++w) {
        const mpmc_status s = run_sweeps(h, window_sweeps);
        if (s) return s;
        MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
        MPMC_HIP(mpmc::launch_tune(h->t, 1, h->st));
    }
    return MPMC_OK;
}

mpmc_status mpmc_set_launch(mpmc_handle h, int32_t lanes_per_cell, int32_t block_size)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (lanes_per_cell != 1 && lanes_per_cell != 2 && lanes_per_cell != 4 && lanes_per_cell != 64)
        return fail(MPMC_EINVAL, "lanes_per_cell must be 1, 2, 4 or 64");
    if (block_size < 64 || block_size > 256 || block_size % 64)
        return fail(MPMC_EINVAL, "block size must be a multiple of 64 in [64, 256]");
    if (block_size != h->block || lanes_per_cell != h->lanes) drop_graphs(h);
    h->block = block_size;
    h->lanes = lanes_per_cell;
    return MPMC_OK;
}

mpmc_status mpmc_set_sweep_kernel(mpmc_handle h, int32_t fused)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    const bool f = fused != 0;
    if (f != h->fused) drop_graphs(h);
    h->fused = f;
    return MPMC_OK;
}

mpmc_status mpmc_get_sweep_kernel(mpmc_handle h, int32_t *fused)
{
    if (!h || !fused) return fail(MPMC_EINVAL, "null argument");
    *fused = use_fused(h) ? 1 : 0;
    return MPMC_OK;
}

mpmc_status mpmc_get_fused_tile(mpmc_handle h, int32_t *tile, int32_t *tx, int32_t *ty)
{
    if (!h || !tile || !tx || !ty) return fail(MPMC_EINVAL, "null argument");
    const bool f = use_fused(h);
    *tile = f ? h->t.ftile : 0;
    *tx = f ? h->t.ftx : 0;
    *ty = f ? h->t.fty : 0;
    return MPMC_OK;
}

mpmc_status mpmc_autotune(mpmc_handle h, int32_t sweeps, int32_t *lanes_out, int32_t *block_out,
                          double *us_per_sweep_out)
{
    if (!h || sweeps < 16) return fail(MPMC_EINVAL, "autotune needs at least 16 sweeps per candidate");
    MPMC_NEED_STATE(h);
    if (!h->st) return fail(MPMC_EINVAL, "autotune needs a non-default stream");
    hipEvent_t e0, e1;
    MPMC_HIP(hipEventCreate(&e0));
    MPMC_HIP(hipEventCreate(&e1));
    int best_b = h->block, best_l = h->lanes;
    float best_ms = -1.0f;
    mpmc_status s = MPMC_OK;
    for (int l : {1, 2, 4}) {
        for (int b : {64, 128, 192, 256}) {
            s = mpmc_set_launch(h, l, b);
            if (s) break;
            s = run_sweeps(h, sweeps);   // capture and warm
            if (s) break;
            float ms = 0.0f;
            if (hipEventRecord(e0, h->st) != hipSuccess || (s = run_sweeps(h, sweeps)) != MPMC_OK ||
                hipEventRecord(e1, h->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                if (!s) s = fail(MPMC_EHIP, "autotune timing failed");
                break;
            }
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best_b = b;
                best_l = l;
            }
        }
        if (s) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    s = mpmc_set_launch(h, best_l, best_b);
    if (s) return s;
    if (lanes_out) *lanes_out = best_l;
    if (block_out) *block_out = best_b;
    if (us_per_sweep_out) *us_per_sweep_out = 1e3 * (double)best_ms / (double)sweeps;
    return read_ctl(h);
}

mpmc_status mpmc_batch_stats(mpmc_handle h, uint64_t *trials, uint64_t *accepts, float *delta,
                             double *msd)
{
    MPMC_NEED_STATE(h);
    if (msd) {
        if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
        MPMC_HIP(mpmc::launch_msd_all(h->t, h->acc[h->cur], h->count[h->cur], h->st));
    }
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    for (int r = 0; r < h->R(); ++r) {
        const Ctl &c = h->ctl_host[(size_t)r];
        if (trials) trials[r] = c.trials;
        if (accepts) accepts[r] = c.accepts;
        if (delta) delta[r] = c.delta;
        if (msd) msd[r] = c.msd;
    }
    return MPMC_OK;
}

mpmc_status mpmc_control(mpmc_handle h, const float *W, int32_t window_sweeps, int32_t n_windows)
{
    if (!h || !W || window_sweeps < 1 || n_windows < 0)
        return fail(MPMC_EINVAL, "bad controller arguments");
    MPMC_NEED_STATE(h);
    MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
    MPMC_HIP(mpmc::launch_control(h->t, W, 0, h->st));   // open the first window
    for (int w = 0; w < n_windows; ++w) {
        const mpmc_status s = run_sweeps(h, window_sweeps);
        if (s) return s;
        MPMC_HIP(mpmc::launch_fold_counters(h->t, h->work, h->st));
        MPMC_HIP(mpmc::launch_control(h->t, W, 1, h->st));
    }
    return MPMC_OK;
}

mpmc_status mpmc_mlp_work_bytes(int32_t n, size_t *bytes)
{
    if (n < 0 || !bytes) return fail(MPMC_EINVAL, "bad sample count");
    *bytes = mpmc::mlp_work_bytes(n);
    return MPMC_OK;
}

mpmc_status mpmc_mlp_forward(const float *W, const float *X, int32_t n, float *Y, float *cache,
                             void *stream)
{
    if (n < 0 || !W || (n > 0 && (!X || !Y))) return fail(MPMC_EINVAL, "bad forward arguments");
    MPMC_HIP(mpmc::launch_mlp_forward(W, X, n, Y, cache, (hipStream_t)stream));
    return MPMC_OK;
}

mpmc_status mpmc_mlp_backward(const float *W, const float *X, const float *cache, const float *dY,
                              int32_t n, float *dW, float *dX, void *work, void *stream)
{
    if (n < 0 || !W || !dW || !work || (n > 0 && (!X || !cache || !dY)))
        return fail(MPMC_EINVAL, "bad backward arguments");
    MPMC_HIP(mpmc::launch_mlp_backward(W, X, cache, dY, n, dW, dX, work, (hipStream_t)stream));
    return MPMC_OK;
}

mpmc_status mpmc_mlp_backward_noalloc(const float *W, const float *X, const float *cache,
                                      const float *dY, int32_t n, float *dW, float *dX,
                                      void *stream)
{
    if (n < 0 || !W || !dW || (n > 0 && (!X || !cache || !dY)))
        return fail(MPMC_EINVAL, "bad backward arguments");
    if (n > MPMC_MLP_NOALLOC_MAX_SAMPLES)
        return fail(MPMC_EINVAL, "mpmc_mlp_backward_noalloc: n exceeds MPMC_MLP_NOALLOC_MAX_SAMPLES");
    MPMC_HIP(mpmc::launch_mlp_backward_noalloc(W, X, cache, dY, n, dW, dX, (hipStream_t)stream));
    return MPMC_OK;
}

mpmc_status mpmc_mlp_mse(const float *Y, const float *T, int32_t n, float *dY, double *loss,
                         void *work, void *stream)
{
    if (n < 0 || !loss || !work || (n > 0 && (!Y || !T || !dY)))
        return fail(MPMC_EINVAL, "bad loss arguments");
    MPMC_HIP(mpmc::launch_mse(Y, T, n, dY, loss, work, (hipStream_t)stream));
    return MPMC_OK;
}

mpmc_status mpmc_adam_step(float *W, float *m, float *v, const float *dW, int32_t n_params,
                           float lr, float b1, float b2, float eps, int32_t step, void *stream)
{
    if (n_params < 0 || step < 1 || (n_params > 0 && (!W || !m || !v || !dW)))
        return fail(MPMC_EINVAL, "bad Adam arguments");
    if (!(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f && eps > 0.0f && lr >= 0.0f))
        return fail(MPMC_EINVAL, "Adam hyper-parameters out of range");
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, (double)step));
    MPMC_HIP(mpmc::launch_adam(W, m, v, dW, n_params, lr, b1, b2, eps, (float)c1, (float)c2,
                               (hipStream_t)stream));
    return MPMC_OK;
}

mpmc_status mpmc_synchronize(mpmc_handle h)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    return read_ctl(h);
}

void mpmc_destroy(mpmc_handle h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->st);
    drop_graphs(h);
    delete h;
}

}  // extern "C"
