// Host side of libmpmc.so: the C ABI declared in include/mpmc.h.
//
// Validates arguments and geometry, builds the initial lattice, owns no device
// memory (the caller's buffers are used through non-owning pointers), and
// enqueues the kernels of mpmc_kernels.hip on the caller's stream.  Long runs
// of sweeps are captured once into hipGraphs of a fixed, even number of
// sweeps (the ping-pong buffers return to the same half after each graph).
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
constexpr int kRebinBlock = 256;   // workgroup size of the rebin kernels

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

mpmc_status check_params(const mpmc_params *p, const mpmc_geometry &g)
{
    if (!(p->delta > 0.0f) || p->delta > 0.5f * std::min(g.w_x, g.w_y))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    if (p->n_moves < 0 || p->n_moves > (1 << 20)) return fail(MPMC_EINVAL, "n_moves out of range");
    if (p->flags & ~(MPMC_FLAG_ACC | MPMC_FLAG_TAG)) return fail(MPMC_EINVAL, "unknown flag");
    return MPMC_OK;
}

size_t work_bytes(long long C)
{
    return align256((size_t)mpmc::scan_partials(C) * 4) +
           align256((size_t)mpmc::count_stride(C) * 10 * 4) +
           (size_t)mpmc::kMsdBlocksMax * sizeof(double) + 256;
}

}  // namespace

struct mpmc_system {
    mpmc_params p;
    mpmc_geometry geo;
    Geom g;
    hipStream_t st;
    float2 *pos[2];
    uint32_t *start[2];
    float2 *acc[2];
    uint32_t *tag[2];
    mpmc::Work work;
    Ctl *ctl;
    int cur;
    int lanes;
    int block;
    uint32_t key0;
    bool ready;        // a valid, overlap-free state is on the device
    bool lone_pending; // lone sub-sweep counts not yet folded into ctl
    hipGraphExec_t graph[2];
};

namespace {

void drop_graphs(mpmc_system *h)
{
    for (int i = 0; i < 2; ++i)
        if (h->graph[i]) {
            (void)hipGraphExecDestroy(h->graph[i]);
            h->graph[i] = nullptr;
        }
}

mpmc_status read_ctl(mpmc_system *h, Ctl *out)
{
    if (h->lone_pending) {
        MPMC_HIP(mpmc::launch_fold_lone(h->work, h->ctl, h->st));
        h->lone_pending = false;
    }
    MPMC_HIP(hipMemcpyAsync(out, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->st));
    MPMC_HIP(hipStreamSynchronize(h->st));
    if (out->errword) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "device invariant violated (error word 0x%x)%s", out->errword,
                      (out->errword & mpmc::kErrCapacity) ? ": cell above capacity" : "");
        return fail(MPMC_EDEVICE, buf);
    }
    return MPMC_OK;
}

mpmc_status enqueue_subsweep(mpmc_system *h, int set)
{
    if (set >= 0) h->lone_pending = true;
    MPMC_HIP(mpmc::launch_subsweep(h->g, h->pos[h->cur], h->start[h->cur], h->acc[h->cur],
                                   h->tag[h->cur], h->ctl, h->work, h->p.n_moves, set, h->lanes,
                                   h->block, h->st));
    return MPMC_OK;
}

// fold_block > 0: the four sub-sweeps of this sweep ran with that workgroup
// size and their counters are folded by the rebin's scan.
mpmc_status enqueue_rebin(mpmc_system *h, int f, float d, int advance, int fold_block)
{
    const int o = h->cur ^ 1;
    MPMC_HIP(mpmc::launch_rebin(h->g, h->pos[h->cur], h->start[h->cur], h->acc[h->cur],
                                h->tag[h->cur], h->pos[o], h->start[o], h->acc[o], h->tag[o],
                                h->work, h->ctl, f, d, advance, kRebinBlock, fold_block, h->st));
    h->cur = o;
    return MPMC_OK;
}

mpmc_status enqueue_sweep(mpmc_system *h)
{
    for (int slot = 0; slot < 4; ++slot) {
        const mpmc_status s = enqueue_subsweep(h, -1 - slot);
        if (s) return s;
    }
    return enqueue_rebin(h, -1, 0.0f, 1, h->block);
}

mpmc_status run_sweeps(mpmc_system *h, int64_t n)
{
    if (h->st) {
        while (n >= kGraphSweeps) {
            hipGraphExec_t &ex = h->graph[h->cur];
            if (!ex) {
                const int cur0 = h->cur;
                hipGraph_t graph = nullptr;
                MPMC_HIP(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
                mpmc_status s = MPMC_OK;
                for (int k = 0; k < kGraphSweeps && s == MPMC_OK; ++k) s = enqueue_sweep(h);
                const hipError_t e = hipStreamEndCapture(h->st, &graph);
                h->cur = cur0;
                if (s) return s;
                if (e != hipSuccess) return fail(MPMC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
                const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ei != hipSuccess) {
                    ex = nullptr;
                    return fail(MPMC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
                }
            }
            MPMC_HIP(hipGraphLaunch(ex, h->st));
            n -= kGraphSweeps;
        }
    }
    for (; n > 0; --n) {
        const mpmc_status s = enqueue_sweep(h);
        if (s) return s;
    }
    return MPMC_OK;
}

mpmc_status validate_host_state(const mpmc_system *h, const float *xy, const uint32_t *start)
{
    const int C = h->g.C;
    if (start[0] != 0) return fail(MPMC_ESTATE, "start[0] != 0");
    for (int c = 0; c < C; ++c) {
        if (start[c + 1] < start[c]) return fail(MPMC_ESTATE, "offsets decrease");
        if (start[c + 1] - start[c] > (uint32_t)h->g.cap) return fail(MPMC_ESTATE, "cell above capacity");
    }
    if ((long long)start[C] != h->g.N) return fail(MPMC_ESTATE, "particle count differs from the buffers' N");
    for (long long k = 0; k < h->g.N; ++k) {
        const float x = xy[2 * k], y = xy[2 * k + 1];
        if (!(x > 0.0f && x <= h->g.wx && y > 0.0f && y <= h->g.wy))
            return fail(MPMC_ESTATE, "local coordinate outside (0, w]");
    }
    return MPMC_OK;
}

mpmc_status upload_state(mpmc_system *h, const float *xy, const uint32_t *start, uint64_t sweep,
                         const uint32_t *tags)
{
    const long long N = h->g.N;
    const int C = h->g.C;
    drop_graphs(h);
    h->cur = 0;
    h->ready = false;
    MPMC_HIP(hipMemcpyAsync(h->pos[0], xy, sizeof(float2) * (size_t)N, hipMemcpyHostToDevice, h->st));
    MPMC_HIP(hipMemcpyAsync(h->start[0], start, sizeof(uint32_t) * (size_t)(C + 1), hipMemcpyHostToDevice, h->st));
    std::vector<uint32_t> idx;
    if (h->tag[0]) {
        if (!tags) {
            idx.resize((size_t)N);
            for (long long k = 0; k < N; ++k) idx[(size_t)k] = (uint32_t)k;
            tags = idx.data();
        }
        MPMC_HIP(hipMemcpyAsync(h->tag[0], tags, sizeof(uint32_t) * (size_t)N, hipMemcpyHostToDevice, h->st));
    }
    if (h->acc[0]) MPMC_HIP(mpmc::launch_fill_u32((uint32_t *)h->acc[0], 0u, 2 * N, h->st));
    MPMC_HIP(mpmc::launch_ctl_reset(h->g, h->ctl, sweep, h->key0, h->p.replica, h->p.delta, h->st));
    MPMC_HIP(mpmc::launch_fill_u32(h->work.cnt, 0u, 10LL * h->work.cnt_stride, h->st));
    h->lone_pending = false;
    MPMC_HIP(hipStreamSynchronize(h->st));
    // overlap check in the kernels' metric
    MPMC_HIP(mpmc::launch_count_overlaps(h->g, h->pos[0], h->start[0], h->ctl, h->block, h->st));
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    if (c.overlaps != 0) return fail(MPMC_EOVERLAP, "state contains overlapping disks");
    h->ready = true;
    return MPMC_OK;
}

#define MPMC_NEED_STATE(h)                                                                   \
    do {                                                                                     \
        if (!(h)) return fail(MPMC_EINVAL, "null handle");                                   \
        if (!(h)->ready) return fail(MPMC_ESTATE, "no valid state loaded (mpmc_set_state)"); \
    } while (0)

}  // namespace

extern "C" {

const char *mpmc_last_error(void) { return g_last_error.c_str(); }

mpmc_status mpmc_geometry_of(const mpmc_params *p, mpmc_geometry *out)
{
    return derive_geometry(p, out);
}

mpmc_status mpmc_required_bytes(const mpmc_params *p, mpmc_buffer_sizes *out)
{
    if (!out) return fail(MPMC_EINVAL, "null argument");
    mpmc_geometry g;
    const mpmc_status s = derive_geometry(p, &g);
    if (s) return s;
    const long long N = g.n_particles, C = (long long)g.cells_x * g.cells_y;
    out->pos = align256(std::max<size_t>(8 * (size_t)N, 8));
    out->start = align256(4 * (size_t)(C + 1));
    out->acc = (p->flags & MPMC_FLAG_ACC) ? align256(std::max<size_t>(8 * (size_t)N, 8)) : 0;
    out->tag = (p->flags & MPMC_FLAG_TAG) ? align256(std::max<size_t>(4 * (size_t)N, 4)) : 0;
    out->work = work_bytes(C);
    out->ctl = align256(sizeof(Ctl));
    return MPMC_OK;
}

mpmc_status mpmc_init_system(const mpmc_params *p, const mpmc_buffers *b, void *stream,
                             mpmc_handle *out)
{
    if (!p || !b || !out) return fail(MPMC_EINVAL, "null argument");
    *out = nullptr;
    mpmc_geometry geo;
    mpmc_status s = derive_geometry(p, &geo);
    if (s) return s;
    s = check_params(p, geo);
    if (s) return s;
    for (int i = 0; i < 2; ++i) {
        if (!b->pos[i] || !b->start[i]) return fail(MPMC_EINVAL, "pos/start buffers missing");
        if ((p->flags & MPMC_FLAG_ACC) && !b->acc[i]) return fail(MPMC_EINVAL, "acc buffers missing");
        if ((p->flags & MPMC_FLAG_TAG) && !b->tag[i]) return fail(MPMC_EINVAL, "tag buffers missing");
    }
    if (!b->work || !b->ctl) return fail(MPMC_EINVAL, "work/ctl buffers missing");

    mpmc_system *h = new mpmc_system();
    h->p = *p;
    h->geo = geo;
    h->g.mx = geo.cells_x;
    h->g.my = geo.cells_y;
    h->g.C = geo.cells_x * geo.cells_y;
    h->g.cap = geo.capacity;
    h->g.wx = geo.w_x;
    h->g.wy = geo.w_y;
    h->g.N = geo.n_particles;
    h->st = (hipStream_t)stream;
    for (int i = 0; i < 2; ++i) {
        h->pos[i] = (float2 *)b->pos[i];
        h->start[i] = (uint32_t *)b->start[i];
        h->acc[i] = (p->flags & MPMC_FLAG_ACC) ? (float2 *)b->acc[i] : nullptr;
        h->tag[i] = (p->flags & MPMC_FLAG_TAG) ? (uint32_t *)b->tag[i] : nullptr;
    }
    {
        char *w = (char *)b->work;
        h->work.scan = (uint32_t *)w;
        w += align256((size_t)mpmc::scan_partials(h->g.C) * 4);
        h->work.cnt = (uint32_t *)w;
        h->work.cnt_stride = (int)mpmc::count_stride(h->g.C);
        w += align256((size_t)mpmc::count_stride(h->g.C) * 10 * 4);
        h->work.f64 = (double *)w;
    }
    h->ctl = (Ctl *)b->ctl;
    h->cur = 0;
    h->lanes = 1;
    h->block = 256;
    h->key0 = p->seed;
    h->ready = false;
    h->lone_pending = false;
    h->graph[0] = h->graph[1] = nullptr;

    const int C = h->g.C;
    const long long N = h->g.N;
    std::vector<uint32_t> start((size_t)C + 1, 0);
    std::vector<float> xy(2 * (size_t)std::max(N, 1LL));
    std::vector<uint32_t> tags((size_t)std::max(N, 1LL));
    if (p->lattice_nx > 0) {
        // Initial condition: lattice site (i, j) at x = (i + 1/4 + (j odd)/2) a,
        // y = (j + 1/2) h in FP64; cell ceil(x/w) - 1; local (float)(x - c w);
        // cells list their disks in ascending lattice index.
        const int nx = p->lattice_nx, ny = p->lattice_ny;
        const Lattice L = lattice_of(nx, ny, p->phi);
        std::vector<int> cell_of((size_t)N);
        std::vector<float> lx((size_t)N), ly((size_t)N);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t k = (size_t)j * nx + i;
                const double x = ((double)i + 0.25 + 0.5 * (double)(j & 1)) * L.a;
                const double y = ((double)j + 0.5) * L.h;
                const int cx = (int)std::ceil(x / (double)h->g.wx) - 1;
                const int cy = (int)std::ceil(y / (double)h->g.wy) - 1;
                if (cx < 0 || cx >= h->g.mx || cy < 0 || cy >= h->g.my) {
                    delete h;
                    return fail(MPMC_EGEOM, "lattice site outside the cell grid");
                }
                lx[k] = (float)(x - (double)cx * (double)h->g.wx);
                ly[k] = (float)(y - (double)cy * (double)h->g.wy);
                cell_of[k] = cy * h->g.mx + cx;
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
        s = validate_host_state(h, xy.data(), start.data());
        if (s) {
            delete h;
            return s;
        }
        s = upload_state(h, xy.data(), start.data(), 0, tags.data());
    } else {
        if (N != 0) {
            // empty until mpmc_set_state; start all zero is not a valid N > 0
            // state, so only the control block is initialised here
            MPMC_HIP(mpmc::launch_ctl_reset(h->g, h->ctl, 0, h->key0, p->replica, p->delta, h->st));
            MPMC_HIP(hipStreamSynchronize(h->st));
            s = MPMC_OK;
        } else {
            s = upload_state(h, xy.data(), start.data(), 0, nullptr);
        }
    }
    if (s) {
        delete h;
        return s;
    }
    *out = h;
    return MPMC_OK;
}

mpmc_status mpmc_sweep(mpmc_handle h, int64_t n_sweeps, uint32_t seed)
{
    if (!h || n_sweeps < 0) return fail(MPMC_EINVAL, "bad handle or sweep count");
    MPMC_NEED_STATE(h);
    if (seed != h->key0) {
        MPMC_HIP(mpmc::launch_ctl_set_key0(h->g, h->ctl, seed, h->st));
        h->key0 = seed;
    }
    return run_sweeps(h, n_sweeps);
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
    if (f >= 0) {
        const float w = f < 2 ? h->g.wx : h->g.wy;
        if (!(d >= 0.0f && d <= 0.5f * w)) return fail(MPMC_EINVAL, "d must lie in [0, w/2]");
    }
    MPMC_NEED_STATE(h);
    if (f >= 0) return enqueue_rebin(h, f, d, 0, 0);
    return enqueue_rebin(h, -1, 0.0f, 1, 0);
}

mpmc_status mpmc_pair_histogram(mpmc_handle h, int32_t reset)
{
    MPMC_NEED_STATE(h);
    if (!h) return fail(MPMC_EINVAL, "null handle");
    const double rmax = 1.0 + MPMC_HIST_BINS * 1e-4;
    const int Rx = (double)h->g.wx >= rmax ? 1 : 2, Ry = (double)h->g.wy >= rmax ? 1 : 2;
    if (h->g.mx < 2 * Rx + 2 || h->g.my < 2 * Ry + 2)
        return fail(MPMC_EGEOM, "grid too small for the histogram's reach");
    MPMC_HIP(mpmc::launch_pair_histogram(h->g, h->pos[h->cur], h->start[h->cur], h->ctl, reset,
                                         h->block, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_pressure_from_contact(mpmc_handle h, double *p_star, double *g_contact,
                                       uint64_t *hist, uint64_t *n_samples)
{
    MPMC_NEED_STATE(h);
    if (!h) return fail(MPMC_EINVAL, "null handle");
    Ctl c;
    mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    if (c.hist_samples == 0) {
        s = mpmc_pair_histogram(h, 1);
        if (s) return s;
    }
    MPMC_HIP(mpmc::launch_pressure_fit(h->g, h->ctl, h->st));
    s = read_ctl(h, &c);
    if (s) return s;
    if (c.fit[3] != 1.0) return fail(MPMC_EDEVICE, "pressure fit failed");
    if (p_star) *p_star = c.fit[0];
    if (g_contact) *g_contact = c.fit[1];
    if (hist) std::memcpy(hist, c.hist, sizeof(c.hist));
    if (n_samples) *n_samples = c.hist_samples;
    return MPMC_OK;
}

mpmc_status mpmc_get_state(mpmc_handle h, float *xy, uint32_t *start, uint64_t *sweep)
{
    MPMC_NEED_STATE(h);
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (xy) MPMC_HIP(hipMemcpyAsync(xy, h->pos[h->cur], sizeof(float2) * (size_t)h->g.N, hipMemcpyDeviceToHost, h->st));
    if (start) MPMC_HIP(hipMemcpyAsync(start, h->start[h->cur], sizeof(uint32_t) * ((size_t)h->g.C + 1), hipMemcpyDeviceToHost, h->st));
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    if (sweep) *sweep = c.sweep;
    return MPMC_OK;
}

mpmc_status mpmc_set_state(mpmc_handle h, const float *xy, const uint32_t *start, uint64_t sweep,
                           const uint32_t *tags)
{
    if (!h || !start || (!xy && h->g.N > 0)) return fail(MPMC_EINVAL, "null argument");
    mpmc_status s = validate_host_state(h, xy, start);
    if (s) return s;
    return upload_state(h, xy, start, sweep, tags);
}

mpmc_status mpmc_get_aux(mpmc_handle h, float *acc, uint32_t *tags)
{
    MPMC_NEED_STATE(h);
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (acc) {
        if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
        MPMC_HIP(hipMemcpyAsync(acc, h->acc[h->cur], sizeof(float2) * (size_t)h->g.N, hipMemcpyDeviceToHost, h->st));
    }
    if (tags) {
        if (!h->tag[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_TAG");
        MPMC_HIP(hipMemcpyAsync(tags, h->tag[h->cur], sizeof(uint32_t) * (size_t)h->g.N, hipMemcpyDeviceToHost, h->st));
    }
    Ctl c;
    return read_ctl(h, &c);
}

mpmc_status mpmc_reset_acc(mpmc_handle h)
{
    MPMC_NEED_STATE(h);
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    MPMC_HIP(mpmc::launch_fill_u32((uint32_t *)h->acc[h->cur], 0u, 2 * h->g.N, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_msd(mpmc_handle h, double *msd)
{
    MPMC_NEED_STATE(h);
    if (!h || !msd) return fail(MPMC_EINVAL, "null argument");
    if (!h->acc[h->cur]) return fail(MPMC_EINVAL, "system built without MPMC_FLAG_ACC");
    MPMC_HIP(mpmc::launch_msd(h->g, h->acc[h->cur], h->work, h->ctl, h->st));
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    *msd = c.msd;
    return MPMC_OK;
}

mpmc_status mpmc_count_overlaps(mpmc_handle h, int64_t *pairs)
{
    MPMC_NEED_STATE(h);
    if (!h || !pairs) return fail(MPMC_EINVAL, "null argument");
    MPMC_HIP(mpmc::launch_count_overlaps(h->g, h->pos[h->cur], h->start[h->cur], h->ctl, h->block, h->st));
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    *pairs = c.overlaps;
    return MPMC_OK;
}

mpmc_status mpmc_get_counters(mpmc_handle h, uint64_t *trials, uint64_t *accepts)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    if (trials) *trials = c.trials;
    if (accepts) *accepts = c.accepts;
    return MPMC_OK;
}

mpmc_status mpmc_set_delta(mpmc_handle h, float delta)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (!(delta > 0.0f) || delta > 0.5f * std::min(h->g.wx, h->g.wy))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    MPMC_HIP(mpmc::launch_ctl_set_delta(h->ctl, delta, h->st));
    h->p.delta = delta;
    return MPMC_OK;
}

mpmc_status mpmc_get_delta(mpmc_handle h, float *delta)
{
    if (!h || !delta) return fail(MPMC_EINVAL, "null argument");
    Ctl c;
    const mpmc_status s = read_ctl(h, &c);
    if (s) return s;
    *delta = c.delta;
    return MPMC_OK;
}

mpmc_status mpmc_tune(mpmc_handle h, int32_t window_sweeps, int32_t n_windows)
{
    if (!h || window_sweeps < 1 || n_windows < 0) return fail(MPMC_EINVAL, "bad tuner arguments");
    MPMC_NEED_STATE(h);
    MPMC_HIP(mpmc::launch_tune(h->g, h->ctl, 0, h->st));   // open the first window
    for (int w = 0; w < n_windows; ++w) {
        const mpmc_status s = run_sweeps(h, window_sweeps);
        if (s) return s;
        MPMC_HIP(mpmc::launch_tune(h->g, h->ctl, 1, h->st));
    }
    return MPMC_OK;
}

mpmc_status mpmc_set_launch(mpmc_handle h, int32_t lanes_per_cell, int32_t block_size)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (lanes_per_cell != 1)
        return fail(MPMC_EINVAL, "lanes_per_cell must be 1");
    if (block_size < 64 || block_size > 256 || block_size % 64)
        return fail(MPMC_EINVAL, "block size must be a multiple of 64 in [64, 256]");
    drop_graphs(h);
    h->lanes = lanes_per_cell;
    h->block = block_size;
    return MPMC_OK;
}

mpmc_status mpmc_autotune(mpmc_handle h, int32_t sweeps, int32_t *block_out,
                          double *us_per_sweep_out)
{
    if (!h || sweeps < 16) return fail(MPMC_EINVAL, "autotune needs at least 16 sweeps per candidate");
    MPMC_NEED_STATE(h);
    if (!h->st) return fail(MPMC_EINVAL, "autotune needs a non-default stream");
    const int candidates[] = {64, 128, 192, 256};
    hipEvent_t e0, e1;
    MPMC_HIP(hipEventCreate(&e0));
    MPMC_HIP(hipEventCreate(&e1));
    int best = h->block;
    float best_ms = -1.0f;
    mpmc_status s = MPMC_OK;
    for (int b : candidates) {
        s = mpmc_set_launch(h, h->lanes, b);
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
            best = b;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    s = mpmc_set_launch(h, h->lanes, best);
    if (s) return s;
    if (block_out) *block_out = best;
    if (us_per_sweep_out) *us_per_sweep_out = 1e3 * (double)best_ms / (double)sweeps;
    Ctl c;
    return read_ctl(h, &c);
}

mpmc_status mpmc_synchronize(mpmc_handle h)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    Ctl c;
    return read_ctl(h, &c);
}

void mpmc_destroy(mpmc_handle h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->st);
    drop_graphs(h);
    delete h;
}

}  // extern "C"
