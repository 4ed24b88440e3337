// Host side of the hard-sphere calls of libmpmc.so (include/mpmc_sphere.h).
//
// Validates arguments and geometry, builds the simple cubic start, owns no
// device memory (the caller's buffers are used through non-owning pointers)
// and enqueues the kernels of sphere_kernels.hip on the caller's stream.
// Long runs of sweeps are captured once into hipGraphs of a fixed, even
// number of sweeps, so the ping-pong buffers return to the same half after
// each graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpmc_sphere.h"
#include "sphere_internal.h"

using mpmc::sph::Ctl3;
using mpmc::sph::Geom3;
using mpmc::sph::kCap;

struct mpmc_sphere {
    Geom3 g;
    mpmc_sphere_params p;
    hipStream_t st;
    float4 *pos[2];
    uint32_t *count[2];
    uint32_t *tag[2];
    float4 *acc[2];
    unsigned long long *cnt;
    double *msd_part;   // per-tile partials of the MSD reduction (in the work buffer)
    Ctl3 *ctl;
    int cur;
    int lanes;   // sub-sweep lanes per active cell
    bool loaded;
    hipGraphExec_t graph[2];
    Ctl3 ctl_host;
};

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kGraphSweeps = 16;   // sweeps per captured graph (even)
constexpr int kDefaultLanes = 1;   // sub-sweep lanes per active cell

// The bits of a uint32 as a float (slot 0's fourth word carries the count).
float u32_as_float(uint32_t u)
{
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

mpmc_status fail(mpmc_status st, const std::string &msg)
{
    mpmc::set_last_error(msg.c_str());
    return st;
}

#define SPH_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(MPMC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Largest width at which at most 8 unit-diameter centres fit in a cube: a
// ninth centre needs w >= 2/sqrt(3); a 1e-5 relative margin covers the FP32
// overlap metric.
double width_limit() { return 2.0 / std::sqrt(3.0) * (1.0 - 1e-5); }

// Lattice spacing of a simple cubic lattice at packing fraction eta:
// eta = (pi/6) / a^3.
double spacing(double eta) { return std::cbrt(kPi / (6.0 * eta)); }

// Smallest even m with L / m < w_max.
int even_cells_below(double L, double w_max)
{
    int m = 2 * (int)std::floor(L / (2.0 * w_max));
    if (m < 2) m = 2;
    while (m > 2 && L / (double)(m - 2) < w_max) m -= 2;
    while (L / (double)m >= w_max) m += 2;
    return m;
}

mpmc_status derive(const mpmc_sphere_params *p, Geom3 &g)
{
    if (!p) return fail(MPMC_EINVAL, "null argument");
    std::memset(&g, 0, sizeof g);
    if (p->flags & ~(uint32_t)(MPMC_FLAG_TAG | MPMC_FLAG_ACC))
        return fail(MPMC_EINVAL, "spheres take no flags but MPMC_FLAG_TAG and MPMC_FLAG_ACC");
    if (p->n_moves < 0 || p->n_moves > (1 << 20)) return fail(MPMC_EINVAL, "n_moves must lie in [0, 2^20]");
    int m[3];
    float w[3];
    if (p->lattice_nx > 0) {
        if (p->lattice_ny < 1 || p->lattice_nz < 1) return fail(MPMC_EINVAL, "lattice sides must be >= 1");
        if (!(p->eta > 0.0 && p->eta <= kPi / 6.0)) return fail(MPMC_EINVAL, "eta must lie in (0, pi/6]");
        const double a = spacing(p->eta);
        const int n3[3] = {p->lattice_nx, p->lattice_ny, p->lattice_nz};
        const int req[3] = {p->cells_x, p->cells_y, p->cells_z};
        const double wm = (p->w_max > 0.0 && p->w_max < width_limit()) ? p->w_max : width_limit();
        for (int k = 0; k < 3; ++k) {
            const double L = (double)n3[k] * a;
            m[k] = req[k] > 0 ? req[k] : even_cells_below(L, wm);
            w[k] = (float)(L / (double)m[k]);
        }
        g.N = (long long)p->lattice_nx * p->lattice_ny * p->lattice_nz;
    } else {
        m[0] = p->cells_x;
        m[1] = p->cells_y;
        m[2] = p->cells_z;
        w[0] = p->cell_w_x;
        w[1] = p->cell_w_y;
        w[2] = p->cell_w_z;
        g.N = p->n_particles;
    }
    for (int k = 0; k < 3; ++k) {
        if (m[k] < 4 || (m[k] & 1)) return fail(MPMC_EGEOM, "cell counts must be even and >= 4");
        if (!((double)w[k] >= 1.0 && (double)w[k] < width_limit()))
            return fail(MPMC_EGEOM, "cell widths must lie in [1, 2/sqrt(3))");
        g.m[k] = m[k];
        g.w[k] = w[k];
    }
    const long long C = (long long)m[0] * m[1] * m[2];
    // the sub-sweep addresses the slot array with 32-bit byte offsets
    if (C * kCap * (long long)sizeof(float4) > 0x7FFFFF00ll)
        return fail(MPMC_EGEOM, "grid too large (at most 2^24 cells)");
    if (g.N < 0 || g.N > C * kCap) return fail(MPMC_EINVAL, "particle count outside [0, 8 cells]");
    if (!(p->delta > 0.0f) || p->delta > 0.5f * std::min(w[0], std::min(w[1], w[2])))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    g.C = (int)C;
    g.active = g.C / 8;
    g.n_moves = p->n_moves;
    return MPMC_OK;
}

// The work buffer: sub-sweep counter partials, then the MSD partials.
size_t counter_bytes(const Geom3 &g)
{
    return align256(2 * sizeof(unsigned long long) * (size_t)mpmc::sph::subsweep_groups(g));
}

void sizes_of(const mpmc_sphere_params *p, const Geom3 &g, mpmc_sphere_buffer_sizes *o)
{
    o->pos = align256(sizeof(float4) * (size_t)g.C * kCap);
    o->count = align256(sizeof(uint32_t) * (size_t)g.C);
    o->tag = (p->flags & MPMC_FLAG_TAG) ? align256(sizeof(uint32_t) * (size_t)g.C * kCap) : 0;
    o->acc = (p->flags & MPMC_FLAG_ACC) ? o->pos : 0;
    const size_t tiles = (size_t)((g.C + mpmc::sph::kTile - 1) / mpmc::sph::kTile);
    o->work = counter_bytes(g) + align256(sizeof(double) * tiles);
    o->ctl = align256(sizeof(Ctl3));
}

void drop_graphs(mpmc_sphere *h)
{
    for (int i = 0; i < 2; ++i)
        if (h->graph[i]) {
            (void)hipGraphExecDestroy(h->graph[i]);
            h->graph[i] = nullptr;
        }
}

// Fold the counter partials, copy the control block, wait, report errors.
mpmc_status read_ctl(mpmc_sphere *h)
{
    SPH_HIP(mpmc::sph::launch_fold3(h->g, h->ctl, h->cnt, h->st));
    SPH_HIP(hipMemcpyAsync(&h->ctl_host, h->ctl, sizeof(Ctl3), hipMemcpyDeviceToHost, h->st));
    SPH_HIP(hipStreamSynchronize(h->st));
    if (h->ctl_host.errword) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "device invariant violated (error word 0x%x)%s",
                      h->ctl_host.errword,
                      (h->ctl_host.errword & mpmc::sph::kErrCapacity) ? ": cell above capacity" : "");
        return fail(MPMC_EDEVICE, buf);
    }
    return MPMC_OK;
}

mpmc_status enqueue_subsweep(mpmc_sphere *h, int set)
{
    SPH_HIP(mpmc::sph::launch_subsweep3(h->g, h->ctl, h->cur, h->pos[h->cur], h->count[h->cur],
                                        h->tag[h->cur], h->acc[h->cur], h->cnt, set, h->lanes,
                                        h->st));
    return MPMC_OK;
}

mpmc_status enqueue_rebin(mpmc_sphere *h, int f, float d)
{
    const int o = h->cur ^ 1;
    SPH_HIP(mpmc::sph::launch_rebin3(h->g, h->ctl, h->cur, h->pos[h->cur], h->count[h->cur],
                                     h->tag[h->cur], h->acc[h->cur], h->pos[o], h->count[o],
                                     h->tag[o], h->acc[o], f, d, h->st));
    h->cur = o;
    return MPMC_OK;
}

mpmc_status enqueue_sweep(mpmc_sphere *h)
{
    for (int slot = 0; slot < 8; ++slot) {
        const mpmc_status s = enqueue_subsweep(h, -1 - slot);
        if (s) return s;
    }
    return enqueue_rebin(h, -1, 0.0f);
}

mpmc_status run_sweeps(mpmc_sphere *h, int64_t n)
{
    if (h->st) {
        while (n >= kGraphSweeps) {
            hipGraphExec_t &ex = h->graph[h->cur];
            if (!ex) {
                const int cur0 = h->cur;
                hipGraph_t graph = nullptr;
                SPH_HIP(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
                mpmc_status s = MPMC_OK;
                for (int k = 0; k < kGraphSweeps && s == MPMC_OK; ++k) s = enqueue_sweep(h);
                const hipError_t e = hipStreamEndCapture(h->st, &graph);
                h->cur = cur0;
                if (s) return s;
                if (e != hipSuccess)
                    return fail(MPMC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
                const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ei != hipSuccess) {
                    ex = nullptr;
                    return fail(MPMC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
                }
            }
            SPH_HIP(hipGraphLaunch(ex, h->st));
            n -= kGraphSweeps;
        }
    }
    for (; n > 0; --n) {
        const mpmc_status s = enqueue_sweep(h);
        if (s) return s;
    }
    return MPMC_OK;
}

mpmc_status validate_host_state(const Geom3 &g, const float *xyz, const uint32_t *start)
{
    if (start[0] != 0) return fail(MPMC_ESTATE, "start[0] != 0");
    for (int c = 0; c < g.C; ++c) {
        if (start[c + 1] < start[c]) return fail(MPMC_ESTATE, "offsets decrease");
        if (start[c + 1] - start[c] > (uint32_t)kCap) return fail(MPMC_ESTATE, "cell above capacity");
    }
    if ((long long)start[g.C] != g.N) return fail(MPMC_ESTATE, "particle count differs from the buffers' N");
    for (long long k = 0; k < g.N; ++k)
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * k + a];
            if (!(v > 0.0f && v <= g.w[a])) return fail(MPMC_ESTATE, "local coordinate outside (0, w]");
        }
    return MPMC_OK;
}

// Compact lists -> slots in the current half, control block reset to
// `sweep`, then the device overlap check.
mpmc_status upload(mpmc_sphere *h, const float *xyz, const uint32_t *start, uint64_t sweep,
                   const uint32_t *tags)
{
    const Geom3 &g = h->g;
    mpmc_status s = validate_host_state(g, xyz, start);
    if (s) return s;
    std::vector<uint32_t> cnt((size_t)g.C, 0u);
    std::vector<float4> slots((size_t)g.C * kCap, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
    std::vector<uint32_t> tg(h->tag[0] ? (size_t)g.C * kCap : 0, 0u);
    for (int c = 0; c < g.C; ++c) {
        const uint32_t b = start[c], n = start[c + 1] - start[c];
        cnt[(size_t)c] = n;
        for (uint32_t i = 0; i < n; ++i) {
            const size_t k = mpmc::sph::slot_of(g.C, c, (int)i), src = (size_t)(b + i);
            slots[k] = make_float4(xyz[3 * src], xyz[3 * src + 1], xyz[3 * src + 2],
                                   i == 0 ? u32_as_float(n) : 0.0f);
            if (!tg.empty()) tg[k] = tags ? tags[src] : (uint32_t)src;
        }
    }
    drop_graphs(h);
    h->cur = 0;
    SPH_HIP(hipMemcpyAsync(h->count[0], cnt.data(), sizeof(uint32_t) * cnt.size(),
                           hipMemcpyHostToDevice, h->st));
    SPH_HIP(hipMemcpyAsync(h->pos[0], slots.data(), sizeof(float4) * slots.size(),
                           hipMemcpyHostToDevice, h->st));
    if (!tg.empty())
        SPH_HIP(hipMemcpyAsync(h->tag[0], tg.data(), sizeof(uint32_t) * tg.size(),
                               hipMemcpyHostToDevice, h->st));
    SPH_HIP(mpmc::sph::launch_ctl_reset3(g, h->ctl, sweep, h->p.seed, h->p.replica, h->p.delta, h->st));
    SPH_HIP(hipMemsetAsync(h->cnt, 0, 2 * sizeof(unsigned long long) * (size_t)mpmc::sph::subsweep_groups(g),
                           h->st));
    if (h->acc[0]) SPH_HIP(mpmc::sph::launch_zero4(h->acc[0], (long long)g.C * kCap, h->st));
    SPH_HIP(mpmc::sph::launch_count_overlaps3(g, h->ctl, h->pos[0], h->count[0], h->st));
    h->loaded = false;
    s = read_ctl(h);
    if (s) return s;
    if (h->ctl_host.overlaps != 0) return fail(MPMC_EOVERLAP, "state contains overlapping spheres");
    h->loaded = true;
    return MPMC_OK;
}

// Simple cubic start: site (i, j, k) at ((i + 1/4) a, (j + 1/4) a,
// (k + 1/4) a) in FP64, cell ceil(x / w) - 1 per axis, local
// (float)(x - cell w) kept inside (0, w]; cells list their spheres in
// ascending lattice index.
mpmc_status build_lattice(const mpmc_sphere_params &p, const Geom3 &g, std::vector<float> &xyz,
                          std::vector<uint32_t> &start, std::vector<uint32_t> &tags)
{
    const int n3[3] = {p.lattice_nx, p.lattice_ny, p.lattice_nz};
    const double a = spacing(p.eta);
    const size_t N = (size_t)g.N;
    std::vector<int> cell_of(N);
    std::vector<float> loc(3 * N);
    start.assign((size_t)g.C + 1, 0u);
    for (int k = 0; k < n3[2]; ++k)
        for (int j = 0; j < n3[1]; ++j)
            for (int i = 0; i < n3[0]; ++i) {
                const size_t id = ((size_t)k * n3[1] + j) * n3[0] + i;
                const int ijk[3] = {i, j, k};
                int cc[3];
                for (int q = 0; q < 3; ++q) {
                    const double x = ((double)ijk[q] + 0.25) * a;
                    int cq = (int)std::ceil(x / (double)g.w[q]) - 1;
                    cq = std::min(std::max(cq, 0), g.m[q] - 1);
                    float l = (float)(x - (double)cq * (double)g.w[q]);
                    if (!(l > 0.0f)) l = std::nextafter(0.0f, 1.0f);
                    if (l > g.w[q]) l = g.w[q];
                    cc[q] = cq;
                    loc[3 * id + q] = l;
                }
                cell_of[id] = (cc[2] * g.m[1] + cc[1]) * g.m[0] + cc[0];
                start[(size_t)cell_of[id] + 1] += 1;
            }
    for (int c = 0; c < g.C; ++c) {
        if (start[(size_t)c + 1] > (uint32_t)kCap) return fail(MPMC_ESTATE, "lattice puts more than 8 spheres in a cell");
        start[(size_t)c + 1] += start[(size_t)c];
    }
    std::vector<uint32_t> fill(start.begin(), start.end() - 1);
    xyz.assign(3 * N, 0.0f);
    tags.assign(N, 0u);
    for (size_t id = 0; id < N; ++id) {
        const uint32_t o = fill[(size_t)cell_of[id]]++;
        for (int q = 0; q < 3; ++q) xyz[3 * (size_t)o + q] = loc[3 * id + q];
        tags[o] = (uint32_t)id;
    }
    return MPMC_OK;
}

#define SPH_NEED_STATE(h)                                                                    \
    do {                                                                                     \
        if (!(h)) return fail(MPMC_EINVAL, "null handle");                                   \
        if (!(h)->loaded) return fail(MPMC_ESTATE, "no valid state loaded (mpmc_sphere_set_state)"); \
    } while (0)

}  // namespace

extern "C" {

mpmc_status mpmc_sphere_geometry_of(const mpmc_sphere_params *p, mpmc_sphere_geometry *out)
{
    if (!out) return fail(MPMC_EINVAL, "null argument");
    Geom3 g;
    const mpmc_status s = derive(p, g);
    if (s) return s;
    out->n_particles = g.N;
    out->cells_x = g.m[0];
    out->cells_y = g.m[1];
    out->cells_z = g.m[2];
    out->w_x = g.w[0];
    out->w_y = g.w[1];
    out->w_z = g.w[2];
    out->box_x = (double)g.m[0] * (double)g.w[0];
    out->box_y = (double)g.m[1] * (double)g.w[1];
    out->box_z = (double)g.m[2] * (double)g.w[2];
    out->density = (double)g.N / (out->box_x * out->box_y * out->box_z);
    return MPMC_OK;
}

mpmc_status mpmc_sphere_required_bytes(const mpmc_sphere_params *p, mpmc_sphere_buffer_sizes *out)
{
    if (!out) return fail(MPMC_EINVAL, "null argument");
    Geom3 g;
    const mpmc_status s = derive(p, g);
    if (s) return s;
    sizes_of(p, g, out);
    return MPMC_OK;
}

mpmc_status mpmc_sphere_init(const mpmc_sphere_params *p, const mpmc_sphere_buffers *b,
                             void *stream, mpmc_sphere_handle *out)
{
    if (!p || !b || !out) return fail(MPMC_EINVAL, "null argument");
    *out = nullptr;
    Geom3 g;
    mpmc_status s = derive(p, g);
    if (s) return s;
    const bool want_tag = (p->flags & MPMC_FLAG_TAG) != 0;
    const bool want_acc = (p->flags & MPMC_FLAG_ACC) != 0;
    for (int i = 0; i < 2; ++i) {
        if (!b->pos[i] || !b->count[i] || (want_tag && !b->tag[i]) || (want_acc && !b->acc[i]))
            return fail(MPMC_EINVAL, "missing device buffer");
        if (((uintptr_t)b->pos[i] | (uintptr_t)b->count[i] | (uintptr_t)(want_tag ? b->tag[i] : nullptr) |
             (uintptr_t)(want_acc ? b->acc[i] : nullptr)) & 255u)
            return fail(MPMC_EINVAL, "device buffers must be 256-byte aligned");
    }
    if (!b->work || !b->ctl || (((uintptr_t)b->work | (uintptr_t)b->ctl) & 255u))
        return fail(MPMC_EINVAL, "missing or misaligned work / ctl buffer");
    mpmc_sphere *h = new mpmc_sphere();
    h->g = g;
    h->p = *p;
    h->st = (hipStream_t)stream;
    for (int i = 0; i < 2; ++i) {
        h->pos[i] = (float4 *)b->pos[i];
        h->count[i] = (uint32_t *)b->count[i];
        h->tag[i] = want_tag ? (uint32_t *)b->tag[i] : nullptr;
        h->acc[i] = want_acc ? (float4 *)b->acc[i] : nullptr;
    }
    h->cnt = (unsigned long long *)b->work;
    h->msd_part = (double *)((char *)b->work + counter_bytes(g));
    h->ctl = (Ctl3 *)b->ctl;
    h->cur = 0;
    h->lanes = kDefaultLanes;
    h->loaded = false;
    h->graph[0] = h->graph[1] = nullptr;
    if (p->lattice_nx > 0) {
        std::vector<float> xyz;
        std::vector<uint32_t> start, tags;
        s = build_lattice(*p, g, xyz, start, tags);
        if (!s) s = upload(h, xyz.data(), start.data(), 0, tags.data());
    } else {
        // an empty grid: counts zero, control block reset; set_state loads it
        s = MPMC_OK;
        hipError_t e = hipMemsetAsync(h->count[0], 0, sizeof(uint32_t) * (size_t)g.C, h->st);
        if (e == hipSuccess) e = mpmc::sph::launch_ctl_reset3(g, h->ctl, 0, p->seed, p->replica, p->delta, h->st);
        if (e == hipSuccess)
            e = hipMemsetAsync(h->cnt, 0, 2 * sizeof(unsigned long long) * (size_t)mpmc::sph::subsweep_groups(g), h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) s = fail(MPMC_EHIP, std::string("init: ") + hipGetErrorString(e));
    }
    if (s) {
        delete h;
        return s;
    }
    *out = h;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_sweep(mpmc_sphere_handle h, int64_t n_sweeps)
{
    if (!h || n_sweeps < 0) return fail(MPMC_EINVAL, "bad handle or sweep count");
    SPH_NEED_STATE(h);
    return run_sweeps(h, n_sweeps);
}

mpmc_status mpmc_sphere_subsweep(mpmc_sphere_handle h, int32_t set)
{
    if (!h || set < 0 || set > 7) return fail(MPMC_EINVAL, "set must be 0..7");
    SPH_NEED_STATE(h);
    return enqueue_subsweep(h, set);
}

mpmc_status mpmc_sphere_shift(mpmc_sphere_handle h, int32_t f, float d)
{
    if (!h || f < -1 || f > 5) return fail(MPMC_EINVAL, "f must be -1..5");
    if (f >= 0 && !(d >= 0.0f && d <= 0.5f * h->g.w[f / 2])) return fail(MPMC_EINVAL, "d must lie in [0, w_f/2]");
    SPH_NEED_STATE(h);
    return enqueue_rebin(h, f, f >= 0 ? d : 0.0f);
}

mpmc_status mpmc_sphere_get_state(mpmc_sphere_handle h, float *xyz, uint32_t *start,
                                  uint32_t *tags, uint64_t *sweep)
{
    SPH_NEED_STATE(h);
    if (tags && !h->tag[0]) return fail(MPMC_EINVAL, "tags need MPMC_FLAG_TAG");
    const Geom3 &g = h->g;
    std::vector<uint32_t> cnt((size_t)g.C);
    std::vector<float4> slots((xyz ? (size_t)g.C * kCap : 0));
    std::vector<uint32_t> tg(tags ? (size_t)g.C * kCap : 0);
    SPH_HIP(hipMemcpyAsync(cnt.data(), h->count[h->cur], sizeof(uint32_t) * cnt.size(),
                           hipMemcpyDeviceToHost, h->st));
    if (xyz)
        SPH_HIP(hipMemcpyAsync(slots.data(), h->pos[h->cur], sizeof(float4) * slots.size(),
                               hipMemcpyDeviceToHost, h->st));
    if (tags)
        SPH_HIP(hipMemcpyAsync(tg.data(), h->tag[h->cur], sizeof(uint32_t) * tg.size(),
                               hipMemcpyDeviceToHost, h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    uint64_t total = 0;
    for (int c = 0; c < g.C; ++c) {
        if (cnt[(size_t)c] > (uint32_t)kCap) return fail(MPMC_EDEVICE, "cell above capacity");
        total += cnt[(size_t)c];
    }
    if ((long long)total != g.N) return fail(MPMC_EDEVICE, "cell counts do not add up to N");
    uint32_t k = 0;
    for (int c = 0; c < g.C; ++c) {
        if (start) start[c] = k;
        for (uint32_t i = 0; i < cnt[(size_t)c]; ++i, ++k) {
            const size_t sl = mpmc::sph::slot_of(g.C, c, (int)i);
            if (xyz) {
                xyz[3 * (size_t)k] = slots[sl].x;
                xyz[3 * (size_t)k + 1] = slots[sl].y;
                xyz[3 * (size_t)k + 2] = slots[sl].z;
            }
            if (tags) tags[k] = tg[sl];
        }
    }
    if (start) start[g.C] = k;
    if (sweep) *sweep = h->ctl_host.sweep_at[h->cur];
    return MPMC_OK;
}

mpmc_status mpmc_sphere_set_state(mpmc_sphere_handle h, const float *xyz, const uint32_t *start,
                                  uint64_t sweep, const uint32_t *tags)
{
    if (!h || !start || (!xyz && h->g.N > 0)) return fail(MPMC_EINVAL, "null argument");
    return upload(h, xyz, start, sweep, tags);
}

mpmc_status mpmc_sphere_get_counters(mpmc_sphere_handle h, uint64_t *trials, uint64_t *accepts)
{
    SPH_NEED_STATE(h);
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    if (trials) *trials = h->ctl_host.trials;
    if (accepts) *accepts = h->ctl_host.accepts;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_set_delta(mpmc_sphere_handle h, float delta)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    if (!(delta > 0.0f) || delta > 0.5f * std::min(h->g.w[0], std::min(h->g.w[1], h->g.w[2])))
        return fail(MPMC_EINVAL, "delta must lie in (0, min(w)/2]");
    SPH_HIP(mpmc::sph::launch_set_delta3(h->ctl, delta, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_sphere_get_delta(mpmc_sphere_handle h, float *delta)
{
    if (!h || !delta) return fail(MPMC_EINVAL, "null argument");
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    *delta = h->ctl_host.delta;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_tune(mpmc_sphere_handle h, int32_t window_sweeps, int32_t n_windows)
{
    if (!h || window_sweeps < 1 || n_windows < 0) return fail(MPMC_EINVAL, "bad tuner arguments");
    SPH_NEED_STATE(h);
    SPH_HIP(mpmc::sph::launch_fold3(h->g, h->ctl, h->cnt, h->st));
    SPH_HIP(mpmc::sph::launch_tune3(h->g, h->ctl, 0, h->st));   // open the first window
    for (int w = 0; w < n_windows; ++w) {
        const mpmc_status s = run_sweeps(h, window_sweeps);
        if (s) return s;
        SPH_HIP(mpmc::sph::launch_fold3(h->g, h->ctl, h->cnt, h->st));
        SPH_HIP(mpmc::sph::launch_tune3(h->g, h->ctl, 1, h->st));
    }
    return MPMC_OK;
}

mpmc_status mpmc_sphere_pair_histogram(mpmc_sphere_handle h, int32_t reset)
{
    SPH_NEED_STATE(h);
    const double rmax = 1.0 + MPMC_HIST_BINS * 1e-4;
    for (int a = 0; a < 3; ++a) {
        const int R = (double)h->g.w[a] >= rmax ? 1 : 2;
        if (h->g.m[a] < 2 * R + 2) return fail(MPMC_EGEOM, "grid too small for the histogram's reach");
    }
    SPH_HIP(mpmc::sph::launch_pair_hist3(h->g, h->ctl, h->pos[h->cur], h->count[h->cur], reset, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_sphere_pressure(mpmc_sphere_handle h, double *p_star, double *g_contact,
                                 uint64_t *hist, uint64_t *n_samples)
{
    SPH_NEED_STATE(h);
    mpmc_status s = read_ctl(h);
    if (s) return s;
    if (h->ctl_host.hist_samples == 0) {
        s = mpmc_sphere_pair_histogram(h, 1);
        if (s) return s;
    }
    SPH_HIP(mpmc::sph::launch_pressure_fit3(h->g, h->ctl, h->st));
    s = read_ctl(h);
    if (s) return s;
    const Ctl3 &c = h->ctl_host;
    if (c.fit[3] != 1.0) return fail(MPMC_EDEVICE, "pressure fit failed");
    if (p_star) *p_star = c.fit[0];
    if (g_contact) *g_contact = c.fit[1];
    if (hist) std::memcpy(hist, c.hist, sizeof(c.hist));
    if (n_samples) *n_samples = c.hist_samples;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_count_overlaps(mpmc_sphere_handle h, int64_t *pairs)
{
    SPH_NEED_STATE(h);
    if (!pairs) return fail(MPMC_EINVAL, "null argument");
    SPH_HIP(mpmc::sph::launch_count_overlaps3(h->g, h->ctl, h->pos[h->cur], h->count[h->cur], h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    *pairs = h->ctl_host.overlaps;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_set_launch(mpmc_sphere_handle h, int32_t lanes_per_cell)
{
    if (!h || !(lanes_per_cell == 1 || lanes_per_cell == 2 || lanes_per_cell == 4))
        return fail(MPMC_EINVAL, "lanes per cell must be 1, 2 or 4");
    if (lanes_per_cell != h->lanes) {
        SPH_HIP(hipStreamSynchronize(h->st));
        drop_graphs(h);
        h->lanes = lanes_per_cell;
    }
    return MPMC_OK;
}

mpmc_status mpmc_sphere_get_acc(mpmc_sphere_handle h, float *acc)
{
    SPH_NEED_STATE(h);
    if (!acc) return fail(MPMC_EINVAL, "null argument");
    if (!h->acc[0]) return fail(MPMC_EINVAL, "accumulators need MPMC_FLAG_ACC");
    const Geom3 &g = h->g;
    std::vector<uint32_t> cnt((size_t)g.C);
    std::vector<float4> slots((size_t)g.C * kCap);
    SPH_HIP(hipMemcpyAsync(cnt.data(), h->count[h->cur], sizeof(uint32_t) * cnt.size(),
                           hipMemcpyDeviceToHost, h->st));
    SPH_HIP(hipMemcpyAsync(slots.data(), h->acc[h->cur], sizeof(float4) * slots.size(),
                           hipMemcpyDeviceToHost, h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    size_t k = 0;
    for (int c = 0; c < g.C; ++c) {
        if (cnt[(size_t)c] > (uint32_t)kCap) return fail(MPMC_EDEVICE, "cell above capacity");
        for (uint32_t i = 0; i < cnt[(size_t)c]; ++i, ++k) {
            if ((long long)k >= g.N) return fail(MPMC_EDEVICE, "cell counts exceed N");
            const float4 &v = slots[mpmc::sph::slot_of(g.C, c, (int)i)];
            acc[3 * k] = v.x;
            acc[3 * k + 1] = v.y;
            acc[3 * k + 2] = v.z;
        }
    }
    if ((long long)k != g.N) return fail(MPMC_EDEVICE, "cell counts do not add up to N");
    return MPMC_OK;
}

mpmc_status mpmc_sphere_msd(mpmc_sphere_handle h, double *msd)
{
    SPH_NEED_STATE(h);
    if (!msd) return fail(MPMC_EINVAL, "null argument");
    if (!h->acc[0]) return fail(MPMC_EINVAL, "the MSD needs MPMC_FLAG_ACC");
    SPH_HIP(mpmc::sph::launch_msd3(h->g, h->ctl, h->acc[h->cur], h->count[h->cur], h->msd_part, h->st));
    const mpmc_status s = read_ctl(h);
    if (s) return s;
    *msd = h->ctl_host.msd;
    return MPMC_OK;
}

mpmc_status mpmc_sphere_reset_acc(mpmc_sphere_handle h)
{
    SPH_NEED_STATE(h);
    if (!h->acc[0]) return fail(MPMC_EINVAL, "accumulators need MPMC_FLAG_ACC");
    SPH_HIP(mpmc::sph::launch_zero4(h->acc[h->cur], (long long)h->g.C * kCap, h->st));
    return MPMC_OK;
}

mpmc_status mpmc_sphere_synchronize(mpmc_sphere_handle h)
{
    if (!h) return fail(MPMC_EINVAL, "null handle");
    return read_ctl(h);
}

void mpmc_sphere_destroy(mpmc_sphere_handle h)
{
    if (!h) return;
    drop_graphs(h);
    delete h;
}

}  // extern "C"
