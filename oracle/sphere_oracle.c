/* Serial checkerboard Monte Carlo of hard SPHERES in three dimensions --
 * TEST INFRASTRUCTURE ONLY (the CPU oracle of the 3D chain; the product never
 * links it).
 *
 * The paper states its method for d dimensions (Sec. 2): cells of width
 * w >= sigma, 2^d checkerboard sets processed in random order, each active
 * cell updating only its own particles with trial moves that must stay in
 * the cell and not overlap any particle of the 3^d neighbourhood, then a
 * random shift of the cell grid along one axis (Sec. 3.2).  This file is
 * that chain for d = 3, written plainly and serially:
 *
 *   S1 geometry: an nx x ny x nz simple cubic lattice at packing fraction
 *      eta = N pi / (6 V), spacing a = (pi / (6 eta))^(1/3); cells m_i even
 *      >= 4 with 1 <= w_i < 2/sqrt(3) (then at most 8 centres fit in a cell:
 *      the cube's corners; a ninth needs w >= 2/sqrt(3)), capacity 8;
 *      cell c = (cz m_y + cy) m_x + cx, set Q = (cx&1) + 2(cy&1) + 4(cz&1).
 *   S3 start: site (i, j, k) at ((i + 1/4) a, (j + 1/4) a, (k + 1/4) a) in
 *      FP64, cell ceil(x / w) - 1 per axis, local (float)(x - c w); cells
 *      list their spheres in ascending lattice index (k n_y + j) n_x + i.
 *   S4 random numbers: Philox4x32-10, key (seed, replica), counter (cell,
 *      sweep lo, sweep hi, tag).  Trial t uses words 2(t&1) and 2(t&1)+1 of
 *      trial block t >> 1: x and y from the two halves of the first, z from
 *      the high half of the second; each half h gives the midpoint
 *      (2h + 1 - 65536) / 65536 of one of 65536 parts of (-1, 1), times
 *      delta.  Shuffle draws as in 2D (tag 0x40000000 + b).
 *   S5 sweep s: words u0..u7 of the global blocks (0xFFFFFFFF, s,
 *      0x80000000) and (..., 0x80000001) shuffle the 8 sets (Fisher-Yates,
 *      i = 7..1, j = bounded(u_{7-i}, i + 1)); f = bounded(u7, 6) picks
 *      +x, -x, +y, -y, +z, -z; d = u24 of the first word of block (...,
 *      0x80000002) times w_f / 2.  Sub-sweeps in order, then the shift.
 *   S7 trial: as in 2D with three coordinates; the overlap test is
 *      r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx*ddx)) < 1 over the 27 cells
 *      (ddx*ddx rounded, each further square added by one fused
 *      multiply-add).
 *   S8 shift: as in 2D along the axis of f.
 *   S9 pair histogram: ordered pairs within reach, r^2 bins on FP32 edges
 *      (1 + b 1e-4)^2 computed in FP64.
 *   S10 displacement accumulators: an accepted move adds its displacement
 *      to the sphere's accumulator, one FP32 add per axis; accumulators go
 *      with their sphere through shuffles and shifts and start at zero.
 * Every floating-point operation is one rounded FP32 operation in the order
 * written (compiled with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t oracle_bounded(uint32_t v, uint32_t k);

#define SPH_CAP 8
#define SPH_TAG_SHUFFLE 0x40000000u
#define SPH_TAG_SWEEP 0x80000000u
#define SPH_CELL_GLOBAL 0xFFFFFFFFu
#define SPH_HIST_BINS 200
#define SPH_PI 3.14159265358979323846

enum { SPH_OK = 0, SPH_EINVAL = -1, SPH_EGEOM = -2, SPH_ESTATE = -3 };

typedef struct sphere_sys {
    int m[3];          /* cells per axis */
    float w[3];        /* cell widths */
    int C;
    int64_t N;
    int *n;            /* [C] spheres per cell */
    float *x;          /* [C][SPH_CAP][3] cell-local coordinates */
    uint32_t *tag;     /* [C][SPH_CAP] identity of each sphere */
    int *n2;           /* shift double buffers */
    float *x2;
    uint32_t *tag2;
    float *acc;        /* [C][SPH_CAP][3] displacement accumulated by accepted moves */
    float *acc2;
    float delta;
    int n_moves;
    uint32_t key[2];
    uint64_t sweep;
    uint64_t trials, accepts;
} sphere_sys;

/* Largest cell width that still holds at most 8 centres, with a relative
 * margin against rounding. */
static double sphere_w_limit(void) { return 2.0 / sqrt(3.0) * (1.0 - 1e-5); }

static int wrapi(int v, int m) { return v < 0 ? v + m : (v >= m ? v - m : v); }

static void block(const sphere_sys *S, uint32_t c0, uint64_t s, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, (uint32_t)s, (uint32_t)(s >> 32), tag};
    oracle_philox(ctr, S->key, out);
}

static float half_to_unit(uint32_t h)
{
    return (float)(2 * (int32_t)h + 1 - 65536) * 0x1p-16f;
}

/* S4: the displacement of one trial from its two words. */
void sphere_trial_displacement(uint32_t a, uint32_t b, float delta, float out[3])
{
    out[0] = half_to_unit(a >> 16) * delta;
    out[1] = half_to_unit(a & 0xFFFFu) * delta;
    out[2] = half_to_unit(b >> 16) * delta;
}

static sphere_sys *alloc_sys(const int m[3], const float w[3], int64_t N)
{
    sphere_sys *S = (sphere_sys *)calloc(1, sizeof(sphere_sys));
    if (!S) return NULL;
    memcpy(S->m, m, sizeof S->m);
    memcpy(S->w, w, sizeof S->w);
    S->C = m[0] * m[1] * m[2];
    S->N = N;
    size_t C = (size_t)S->C;
    S->n = (int *)calloc(C, sizeof(int));
    S->n2 = (int *)calloc(C, sizeof(int));
    S->x = (float *)calloc(C * SPH_CAP * 3, sizeof(float));
    S->x2 = (float *)calloc(C * SPH_CAP * 3, sizeof(float));
    S->acc = (float *)calloc(C * SPH_CAP * 3, sizeof(float));
    S->acc2 = (float *)calloc(C * SPH_CAP * 3, sizeof(float));
    S->tag = (uint32_t *)calloc(C * SPH_CAP, sizeof(uint32_t));
    S->tag2 = (uint32_t *)calloc(C * SPH_CAP, sizeof(uint32_t));
    if (!S->n || !S->n2 || !S->x || !S->x2 || !S->tag || !S->tag2 || !S->acc || !S->acc2) {
        free(S->n); free(S->n2); free(S->x); free(S->x2); free(S->tag); free(S->tag2);
        free(S->acc); free(S->acc2);
        free(S);
        return NULL;
    }
    return S;
}

void sphere_destroy(sphere_sys *S)
{
    if (!S) return;
    free(S->n); free(S->n2); free(S->x); free(S->x2); free(S->tag); free(S->tag2);
    free(S->acc); free(S->acc2);
    free(S);
}

static int widths_ok(const float w[3])
{
    for (int a = 0; a < 3; ++a)
        if (!((double)w[a] >= 1.0 && (double)w[a] < sphere_w_limit())) return 0;
    return 1;
}

/* A grid with given cells and widths, every cell empty (for set_state). */
sphere_sys *sphere_create_grid(int mx, int my, int mz, float wx, float wy, float wz, int64_t N,
                               float delta, int n_moves, uint32_t seed, uint32_t replica,
                               int *status)
{
    int m[3] = {mx, my, mz};
    float w[3] = {wx, wy, wz};
    *status = SPH_EGEOM;
    for (int a = 0; a < 3; ++a)
        if (m[a] < 4 || (m[a] & 1)) return NULL;
    if (!widths_ok(w) || N < 0 || N > (int64_t)mx * my * mz * SPH_CAP) return NULL;
    *status = SPH_EINVAL;
    if (!(delta > 0.0f) || n_moves < 0) return NULL;
    sphere_sys *S = alloc_sys(m, w, N);
    if (!S) return NULL;
    S->delta = delta;
    S->n_moves = n_moves;
    S->key[0] = seed;
    S->key[1] = replica;
    *status = SPH_OK;
    return S;
}

/* S1 + S3: the simple cubic lattice at packing fraction eta. */
sphere_sys *sphere_create(int nx, int ny, int nz, double eta, int mx, int my, int mz,
                          double w_max, float delta, int n_moves, uint32_t seed,
                          uint32_t replica, int *status)
{
    *status = SPH_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || !(eta > 0.0) || eta > SPH_PI / 6.0) return NULL;
    const int64_t N = (int64_t)nx * ny * nz;
    const double a = cbrt(SPH_PI / (6.0 * eta));
    const int nn[3] = {nx, ny, nz};
    int m[3] = {mx, my, mz};
    double L[3];
    float w[3];
    const double wm = (w_max > 0.0 && w_max < sphere_w_limit()) ? w_max : sphere_w_limit();
    for (int k = 0; k < 3; ++k) {
        L[k] = (double)nn[k] * a;
        if (m[k] <= 0) {                     /* smallest even m with L/m < w_max */
            int mm = (int)ceil(L[k] / wm);
            if (mm & 1) mm += 1;
            while (L[k] / mm >= wm) mm += 2;
            m[k] = mm;
        }
        w[k] = (float)(L[k] / m[k]);
    }
    sphere_sys *S = sphere_create_grid(m[0], m[1], m[2], w[0], w[1], w[2], N, delta, n_moves,
                                       seed, replica, status);
    if (!S) return NULL;
    /* place the sites, then list each cell's spheres in lattice order */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double p[3] = {(i + 0.25) * a, (j + 0.25) * a, (k + 0.25) * a};
                int c3[3];
                float l[3];
                for (int q = 0; q < 3; ++q) {
                    c3[q] = (int)ceil(p[q] / (double)w[q]) - 1;
                    if (c3[q] < 0) c3[q] = 0;
                    if (c3[q] >= m[q]) c3[q] = m[q] - 1;
                    l[q] = (float)(p[q] - (double)c3[q] * (double)w[q]);
                    if (!(l[q] > 0.0f)) l[q] = nextafterf(0.0f, 1.0f);
                    if (l[q] > w[q]) l[q] = w[q];
                }
                const int c = (c3[2] * m[1] + c3[1]) * m[0] + c3[0];
                if (S->n[c] >= SPH_CAP) {
                    sphere_destroy(S);
                    *status = SPH_ESTATE;
                    return NULL;
                }
                const int s = c * SPH_CAP + S->n[c]++;
                memcpy(&S->x[3 * (size_t)s], l, sizeof l);
                S->tag[s] = (uint32_t)(((int64_t)k * ny + j) * nx + i);
            }
    return S;
}

void sphere_info(const sphere_sys *S, int m[3], float w[3], int64_t *N)
{
    memcpy(m, S->m, sizeof S->m);
    memcpy(w, S->w, sizeof S->w);
    *N = S->N;
}

/* S7 overlap test of a trial position of slot `self` of cell (cx, cy, cz). */
static int overlaps(const sphere_sys *S, const int cc[3], int self, const float xm[3])
{
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                const int o[3] = {ox, oy, oz};
                int nc3[3];
                float tr[3];
                for (int a = 0; a < 3; ++a) {
                    nc3[a] = wrapi(cc[a] + o[a], S->m[a]);
                    tr[a] = o[a] < 0 ? -S->w[a] : (o[a] > 0 ? S->w[a] : 0.0f);
                }
                const int nc = (nc3[2] * S->m[1] + nc3[1]) * S->m[0] + nc3[0];
                const int own = (ox == 0 && oy == 0 && oz == 0);
                for (int j = 0; j < S->n[nc]; ++j) {
                    const int slot = nc * SPH_CAP + j;
                    if (own && slot == self) continue;
                    const float *p = &S->x[3 * (size_t)slot];
                    const float ddx = xm[0] - (p[0] + tr[0]);
                    const float ddy = xm[1] - (p[1] + tr[1]);
                    const float ddz = xm[2] - (p[2] + tr[2]);
                    const float r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                    if (r2 < 1.0f) return 1;
                }
            }
    return 0;
}

static void swap_slots(sphere_sys *S, int a, int b)
{
    float t[3];
    memcpy(t, &S->x[3 * (size_t)a], sizeof t);
    memcpy(&S->x[3 * (size_t)a], &S->x[3 * (size_t)b], sizeof t);
    memcpy(&S->x[3 * (size_t)b], t, sizeof t);
    uint32_t u = S->tag[a];
    S->tag[a] = S->tag[b];
    S->tag[b] = u;
    memcpy(t, &S->acc[3 * (size_t)a], sizeof t);
    memcpy(&S->acc[3 * (size_t)a], &S->acc[3 * (size_t)b], sizeof t);
    memcpy(&S->acc[3 * (size_t)b], t, sizeof t);
}

/* One cell update (the 3D Alg. 2): shuffle the list, then n_M trials on
 * list[t mod n], each kept iff it stays in the cell and overlaps nothing. */
static void cell_update(sphere_sys *S, const int cc[3])
{
    const int c = (cc[2] * S->m[1] + cc[1]) * S->m[0] + cc[0];
    const int n = S->n[c];
    if (n == 0) return;
    const int base = c * SPH_CAP;
    uint32_t wds[4];
    for (int k = 0; k < n - 1; ++k) {
        if ((k & 3) == 0) block(S, (uint32_t)c, S->sweep, SPH_TAG_SHUFFLE + (uint32_t)(k >> 2), wds);
        const int i = n - 1 - k;
        const int j = (int)oracle_bounded(wds[k & 3], (uint32_t)(i + 1));
        swap_slots(S, base + i, base + j);
    }
    for (int t = 0; t < S->n_moves; ++t) {
        if ((t & 1) == 0) block(S, (uint32_t)c, S->sweep, (uint32_t)(t >> 1), wds);
        const int slot = base + t % n;
        float d[3], xm[3];
        sphere_trial_displacement(wds[2 * (t & 1)], wds[2 * (t & 1) + 1], S->delta, d);
        float *p = &S->x[3 * (size_t)slot];
        int in_cell = 1;
        for (int a = 0; a < 3; ++a) {
            xm[a] = p[a] + d[a];
            in_cell = in_cell && xm[a] > 0.0f && xm[a] <= S->w[a];
        }
        S->trials += 1;
        if (in_cell && !overlaps(S, cc, slot, xm)) {
            memcpy(p, xm, sizeof xm);
            float *ac = &S->acc[3 * (size_t)slot];
            for (int a = 0; a < 3; ++a) ac[a] = ac[a] + d[a];
            S->accepts += 1;
        }
    }
}

/* Sub-sweep of set Q.  mode 0 visits the active cells in row-major order,
 * 1 in reverse, 2 in a scrambled order: cells of one set never interact, so
 * the result must not depend on it. */
void sphere_subsweep_order(sphere_sys *S, int Q, int mode)
{
    const int h[3] = {S->m[0] / 2, S->m[1] / 2, S->m[2] / 2};
    const int count = h[0] * h[1] * h[2];
    for (int k = 0; k < count; ++k) {
        int idx = k;
        if (mode == 1) idx = count - 1 - k;
        if (mode == 2) idx = (int)(((int64_t)k * 7919 + 13) % count);   /* 7919 prime */
        const int ix = idx % h[0], iy = (idx / h[0]) % h[1], iz = idx / (h[0] * h[1]);
        const int cc[3] = {2 * ix + (Q & 1), 2 * iy + ((Q >> 1) & 1), 2 * iz + ((Q >> 2) & 1)};
        cell_update(S, cc);
    }
}

void sphere_subsweep(sphere_sys *S, int Q) { sphere_subsweep_order(S, Q, 0); }

/* S5 draws of sweep s. */
void sphere_sweep_draws(const sphere_sys *S, uint64_t s, int order[8], int *f, float *d)
{
    uint32_t u[8], g2[4];
    block(S, SPH_CELL_GLOBAL, s, SPH_TAG_SWEEP, u);
    block(S, SPH_CELL_GLOBAL, s, SPH_TAG_SWEEP + 1u, u + 4);
    block(S, SPH_CELL_GLOBAL, s, SPH_TAG_SWEEP + 2u, g2);
    for (int i = 0; i < 8; ++i) order[i] = i;
    for (int i = 7; i >= 1; --i) {
        const int j = (int)oracle_bounded(u[7 - i], (uint32_t)(i + 1));
        const int t = order[i]; order[i] = order[j]; order[j] = t;
    }
    *f = (int)oracle_bounded(u[7], 6u);
    const float wf = S->w[*f / 2];
    const float ud = (float)(g2[0] & 0xFFFFFFu) * 0x1p-24f;
    *d = ud * (0.5f * wf);
}

/* S8: shift by d along f (0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z). */
int sphere_shift(sphere_sys *S, int f, float d)
{
    if (f < 0 || f > 5) return SPH_EINVAL;
    const int ax = f / 2;
    const int sgn = (f & 1) ? -1 : +1;
    const float w = S->w[ax];
    int bad = 0;
    for (int cz = 0; cz < S->m[2]; ++cz)
        for (int cy = 0; cy < S->m[1]; ++cy)
            for (int cx = 0; cx < S->m[0]; ++cx) {
                const int cc[3] = {cx, cy, cz};
                const int c = (cz * S->m[1] + cy) * S->m[0] + cx;
                int nn3[3] = {cx, cy, cz};
                nn3[ax] = wrapi(cc[ax] + sgn, S->m[ax]);
                const int nc = (nn3[2] * S->m[1] + nn3[1]) * S->m[0] + nn3[0];
                int k = 0;
                for (int pass = 0; pass < 2; ++pass) {
                    const int src = pass == 0 ? c : nc;
                    for (int i = 0; i < S->n[src]; ++i) {
                        const int slot = src * SPH_CAP + i;
                        const float *p = &S->x[3 * (size_t)slot];
                        const float t = sgn > 0 ? p[ax] - d : p[ax] + d;
                        const int stays = t > 0.0f && t <= w;
                        if (pass == 0 ? !stays : stays) continue;
                        if (k >= SPH_CAP) { bad = 1; continue; }
                        float q[3];
                        memcpy(q, p, sizeof q);
                        q[ax] = pass == 0 ? t : (sgn > 0 ? t + w : t - w);
                        memcpy(&S->x2[3 * (size_t)(c * SPH_CAP + k)], q, sizeof q);
                        memcpy(&S->acc2[3 * (size_t)(c * SPH_CAP + k)], &S->acc[3 * (size_t)slot],
                               3 * sizeof(float));
                        S->tag2[c * SPH_CAP + k] = S->tag[slot];
                        ++k;
                    }
                }
                S->n2[c] = k;
            }
    float *tf = S->x; S->x = S->x2; S->x2 = tf;
    tf = S->acc; S->acc = S->acc2; S->acc2 = tf;
    uint32_t *tu = S->tag; S->tag = S->tag2; S->tag2 = tu;
    int *ti = S->n; S->n = S->n2; S->n2 = ti;
    return bad ? SPH_ESTATE : SPH_OK;
}

int sphere_sweep(sphere_sys *S, int64_t n_sweeps)
{
    for (int64_t k = 0; k < n_sweeps; ++k) {
        int order[8], f;
        float d;
        sphere_sweep_draws(S, S->sweep, order, &f, &d);
        for (int i = 0; i < 8; ++i) sphere_subsweep(S, order[i]);
        const int st = sphere_shift(S, f, d);
        if (st) return st;
        S->sweep += 1;
    }
    return SPH_OK;
}

/* Compact state: xyz[N][3] in cell order, start[C + 1]; tags optional. */
void sphere_get_state(const sphere_sys *S, float *xyz, uint32_t *start, uint32_t *tags,
                      uint64_t *sweep)
{
    uint32_t k = 0;
    for (int c = 0; c < S->C; ++c) {
        start[c] = k;
        for (int i = 0; i < S->n[c]; ++i, ++k) {
            memcpy(&xyz[3 * (size_t)k], &S->x[3 * (size_t)(c * SPH_CAP + i)], 3 * sizeof(float));
            if (tags) tags[k] = S->tag[c * SPH_CAP + i];
        }
    }
    start[S->C] = k;
    *sweep = S->sweep;
}

int sphere_set_state(sphere_sys *S, const float *xyz, const uint32_t *start, const uint32_t *tags,
                     uint64_t sweep)
{
    if (start[0] != 0 || (int64_t)start[S->C] != S->N) return SPH_ESTATE;
    for (int c = 0; c < S->C; ++c) {
        if (start[c + 1] < start[c] || start[c + 1] - start[c] > SPH_CAP) return SPH_ESTATE;
        for (uint32_t k = start[c]; k < start[c + 1]; ++k)
            for (int a = 0; a < 3; ++a) {
                const float v = xyz[3 * (size_t)k + a];
                if (!(v > 0.0f && v <= S->w[a])) return SPH_ESTATE;
            }
    }
    for (int c = 0; c < S->C; ++c) {
        S->n[c] = (int)(start[c + 1] - start[c]);
        for (int i = 0; i < S->n[c]; ++i) {
            const uint32_t k = start[c] + (uint32_t)i;
            memcpy(&S->x[3 * (size_t)(c * SPH_CAP + i)], &xyz[3 * (size_t)k], 3 * sizeof(float));
            S->tag[c * SPH_CAP + i] = tags ? tags[k] : k;
        }
    }
    memset(S->acc, 0, sizeof(float) * 3 * SPH_CAP * (size_t)S->C);
    S->sweep = sweep;
    S->trials = S->accepts = 0;
    return SPH_OK;
}

/* Displacement accumulators acc[N][3] in cell (list) order. */
void sphere_get_acc(const sphere_sys *S, float *acc)
{
    size_t k = 0;
    for (int c = 0; c < S->C; ++c)
        for (int i = 0; i < S->n[c]; ++i, ++k)
            memcpy(&acc[3 * k], &S->acc[3 * (size_t)(c * SPH_CAP + i)], 3 * sizeof(float));
}

void sphere_set_delta(sphere_sys *S, float delta) { S->delta = delta; }

float sphere_get_delta(const sphere_sys *S) { return S->delta; }

void sphere_counters(const sphere_sys *S, uint64_t *trials, uint64_t *accepts)
{
    *trials = S->trials;
    *accepts = S->accepts;
}

/* FP64 global coordinates in cell order. */
void sphere_global_positions(const sphere_sys *S, double *xyz)
{
    size_t k = 0;
    for (int cz = 0; cz < S->m[2]; ++cz)
        for (int cy = 0; cy < S->m[1]; ++cy)
            for (int cx = 0; cx < S->m[0]; ++cx) {
                const int cc[3] = {cx, cy, cz};
                const int c = (cz * S->m[1] + cy) * S->m[0] + cx;
                for (int i = 0; i < S->n[c]; ++i, ++k)
                    for (int a = 0; a < 3; ++a)
                        xyz[3 * k + a] = (double)cc[a] * (double)S->w[a] +
                                         (double)S->x[3 * (size_t)(c * SPH_CAP + i) + a];
            }
}

/* S9: ordered pairs with 1 <= r < 1.02, binned on r^2 against FP32 edges. */
void sphere_pair_histogram(const sphere_sys *S, uint64_t hist[SPH_HIST_BINS])
{
    float E[SPH_HIST_BINS + 1];
    for (int b = 0; b <= SPH_HIST_BINS; ++b) {
        const double r = 1.0 + b * 1e-4;
        E[b] = (float)(r * r);
    }
    memset(hist, 0, sizeof(uint64_t) * SPH_HIST_BINS);
    const double rmax = 1.0 + SPH_HIST_BINS * 1e-4;
    int R[3];
    for (int a = 0; a < 3; ++a) R[a] = (double)S->w[a] >= rmax ? 1 : 2;
    for (int cz = 0; cz < S->m[2]; ++cz)
        for (int cy = 0; cy < S->m[1]; ++cy)
            for (int cx = 0; cx < S->m[0]; ++cx) {
                const int cc[3] = {cx, cy, cz};
                const int c = (cz * S->m[1] + cy) * S->m[0] + cx;
                for (int i = 0; i < S->n[c]; ++i) {
                    const int si = c * SPH_CAP + i;
                    const float *p = &S->x[3 * (size_t)si];
                    for (int oz = -R[2]; oz <= R[2]; ++oz)
                        for (int oy = -R[1]; oy <= R[1]; ++oy)
                            for (int ox = -R[0]; ox <= R[0]; ++ox) {
                                const int o[3] = {ox, oy, oz};
                                int nc3[3];
                                float tr[3];
                                for (int a = 0; a < 3; ++a) {
                                    nc3[a] = ((cc[a] + o[a]) % S->m[a] + S->m[a]) % S->m[a];
                                    tr[a] = (float)o[a] * S->w[a];
                                }
                                const int nc = (nc3[2] * S->m[1] + nc3[1]) * S->m[0] + nc3[0];
                                for (int j = 0; j < S->n[nc]; ++j) {
                                    const int sj = nc * SPH_CAP + j;
                                    if (sj == si) continue;
                                    const float *q = &S->x[3 * (size_t)sj];
                                    const float ddx = p[0] - (q[0] + tr[0]);
                                    const float ddy = p[1] - (q[1] + tr[1]);
                                    const float ddz = p[2] - (q[2] + tr[2]);
                                    const float r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
                                    if (r2 < E[0] || r2 >= E[SPH_HIST_BINS]) continue;
                                    int lo = 0, hi = SPH_HIST_BINS;
                                    while (hi - lo > 1) {
                                        const int mid = (lo + hi) / 2;
                                        if (r2 >= E[mid]) lo = mid; else hi = mid;
                                    }
                                    hist[lo] += 1;
                                }
                            }
                }
            }
}

/* Spheres with a neighbour closer than 1 in the chain's own metric (S7). */
int64_t sphere_count_overlaps(const sphere_sys *S)
{
    int64_t bad = 0;
    for (int cz = 0; cz < S->m[2]; ++cz)
        for (int cy = 0; cy < S->m[1]; ++cy)
            for (int cx = 0; cx < S->m[0]; ++cx) {
                const int cc[3] = {cx, cy, cz};
                const int c = (cz * S->m[1] + cy) * S->m[0] + cx;
                for (int i = 0; i < S->n[c]; ++i)
                    bad += overlaps(S, cc, c * SPH_CAP + i, &S->x[3 * (size_t)(c * SPH_CAP + i)]);
            }
    return bad;
}
