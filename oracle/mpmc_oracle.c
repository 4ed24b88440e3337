/*
 * mpmc_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain, serial CPU oracle of the massively parallel Monte Carlo (MPMC)
 * hard-disk chain of Anderson, Jankowski, Grubb, Engel and Glotzer,
 * "Massively parallel Monte Carlo for many-particle simulations on GPUs"
 * (arXiv:1211.1646).  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code with the HIP
 * library; both follow the chain specification written down in the design
 * notes (geometry, Philox streams, FP32 operation order).
 *
 * Structure follows the paper:
 *   - Sec. 3.1 data structures: positions live directly in the cell list,
 *     disk[c][i] with room for n_max particles per cell and a count n[c];
 *     every cell has its own local frame, coordinates in (0,w];
 *     neighbour translations are exactly -w, 0 or +w.
 *   - Sec. 2.2 Alg. 1: a sweep shuffles the four checkerboard sets (Eq. 1),
 *     runs one sub-sweep per set, then draws d and f and shifts the cells.
 *   - Sec. 3.2 Alg. 2: one cell update = shuffle the cell's particles,
 *     then n_M trial moves on particle list[s mod n]; a move is kept iff it
 *     stays in the cell and creates no overlap with the 3x3 neighbourhood.
 *   - Sec. 3.2 Alg. 4: the cell shift gathers, for every new cell, the
 *     stayers of the old cell and then the leavers of the cell in direction
 *     f, into a double buffer; every stay/leave decision is one rounded
 *     value compared against (0,w].
 *
 * Every floating-point step is one IEEE binary32 operation with
 * round-to-nearest-even; compile with -ffp-contract=off (no FMA).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EGEOM (-2)
#define ORC_EOVERLAP (-3)
#define ORC_ESTATE (-6)

#define HIST_BINS 200

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications,
 * with the Weyl key schedule between rounds.
 * ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout: counter (c0, sweep_lo, sweep_hi, tag), key (seed, replica).
 * c0 is the cell index for per-cell draws and 0xFFFFFFFF for the draws that
 * belong to the whole sweep. */
#define TAG_TRIAL 0x00000000u   /* + block index, 4 trial words per block */
#define TAG_SHUFFLE 0x40000000u /* + block index, 4 shuffle words per block */
#define TAG_SWEEP 0x80000000u   /* the sweep-global block */
#define CELL_GLOBAL 0xFFFFFFFFu

static void stream_block(uint32_t c0, uint64_t sweep, uint32_t tag,
                         const uint32_t key[2], uint32_t out[4])
{
    uint32_t ctr[4] = {c0, (uint32_t)sweep, (uint32_t)(sweep >> 32), tag};
    oracle_philox(ctr, key, out);
}

/* Uniform integer in [0,k): the high word of v*k (multiply-shift). */
uint32_t oracle_bounded(uint32_t v, uint32_t k)
{
    return (uint32_t)(((uint64_t)v * (uint64_t)k) >> 32);
}

/* One trial word -> displacement in the square (-delta, delta)^2.
 * High 16 bits give x, low 16 bits give y; each is the midpoint of one of
 * 65536 equal sub-intervals of (-1,1), an exactly representable value, so
 * the proposal is symmetric under (dx,dy) -> (-dx,-dy).  The single rounding
 * is the final multiply by delta. */
void oracle_trial_displacement(uint32_t word, float delta, float *dx, float *dy)
{
    int32_t hx = (int32_t)(word >> 16);
    int32_t hy = (int32_t)(word & 0xFFFFu);
    float ux = (float)(2 * hx + 1 - 65536) * 0x1p-16f;
    float uy = (float)(2 * hy + 1 - 65536) * 0x1p-16f;
    *dx = ux * delta;
    *dy = uy * delta;
}

/* One trial word -> displacement uniform in the disk of radius delta
 * (Alg. 2's inCircle(d), the paper's proposal).
 *
 * The high half hr picks the squared radius as the midpoint (2hr+1)/2^17 of
 * one of 65536 equal sub-intervals of (0,1); its square root is uniform in
 * area.  The low half ha picks the angle (2ha+1) pi / 65536: the top two
 * bits are the quadrant q, the low 14 bits the angle inside it.  Inside a
 * quadrant, angles past pi/4 are taken as the mirror image of an angle below
 * pi/4 (cos and sin swap), so the two series below only ever see
 * 0 < x < pi/4, where their Taylor remainders (order 11 and 12) are below
 * 2e-9, far under FP32 rounding.  Turning by a quadrant only permutes and
 * negates (c, s), exactly, so the words ha and ha ^ 0x8000 give exactly
 * opposite displacements and the proposal is symmetric.  Every step is one
 * FP32 operation (sqrtf is correctly rounded), in the order written. */
static float sin_series(float x, float z)
{
    /* x - x^3/3! + x^5/5! - x^7/7! + x^9/9!, Horner in z = x^2 */
    float p = 0x1.71de3ap-19f * z;   /* 1/9! */
    p = p + -0x1.a01a02p-13f;        /* -1/7! */
    p = p * z;
    p = p + 0x1.111112p-7f;          /* 1/5! */
    p = p * z;
    p = p + -0x1.555556p-3f;         /* -1/3! */
    return x + (x * z) * p;
}

static float cos_series(float z)
{
    /* 1 - x^2/2! + x^4/4! - x^6/6! + x^8/8! - x^10/10! */
    float p = -0x1.27e4fcp-22f * z;  /* -1/10! */
    p = p + 0x1.a01a02p-16f;         /* 1/8! */
    p = p * z;
    p = p + -0x1.6c16c2p-10f;        /* -1/6! */
    p = p * z;
    p = p + 0x1.555556p-5f;          /* 1/4! */
    p = p * z;
    p = p + -0.5f;                   /* -1/2! */
    return 1.0f + z * p;
}

void oracle_disk_displacement(uint32_t word, float delta, float *dx, float *dy)
{
    uint32_t hr = word >> 16;
    uint32_t ha = word & 0xFFFFu;
    uint32_t q = ha >> 14;
    uint32_t j = ha & 0x3FFFu;
    uint32_t m = j < 8192u ? j : 16383u - j;          /* mirror about pi/4 */
    float x = (float)(2u * m + 1u) * 0x1.921fb6p-15f; /* (2m+1) pi / 65536 */
    float z = x * x;
    float sn = sin_series(x, z);
    float cs = cos_series(z);
    float c = j < 8192u ? cs : sn;   /* cos and sin of the angle in the quadrant */
    float s = j < 8192u ? sn : cs;
    float a, b;                      /* turned by q quarter turns */
    switch (q) {
    case 0: a = c; b = s; break;
    case 1: a = -s; b = c; break;
    case 2: a = -c; b = -s; break;
    default: a = s; b = -c; break;
    }
    float rho = sqrtf((float)(2u * hr + 1u) * 0x1p-17f);
    float r = rho * delta;
    *dx = r * a;
    *dy = r * b;
}

/* Particle chosen by trial s of a cell update (Alg. 1): the list is
 * walked from the start and wraps around when n_M > n. */
static int visit_slot(int s, int n) { return s % n; }

void oracle_visit_sequence(int n, int n_moves, int *out)
{
    for (int s = 0; s < n_moves; ++s) out[s] = visit_slot(s, n);
}

/* ------------------------------------------------------------------------
 * Geometry (Sec. 3.1; cell width vs capacity from Fig. 3).
 * ------------------------------------------------------------------------ */

/* Largest number of disk centres (mutual distance >= sigma = 1) that fit in
 * a square of side w: the optimal packings of k points in a square give the
 * thresholds sqrt(2) (5 points, Fig. 3), 6/sqrt(13) (6), (2+sqrt(3))/2 (7)
 * and (sqrt(6)+sqrt(2))/2 (8).  A relative margin of 1e-5 keeps the bound
 * valid for the FP32 overlap metric. */
static int capacity_for_width(double w)
{
    const double margin = 1.0 - 1e-5;
    if (w < sqrt(2.0) * margin) return 4;
    if (w < 6.0 / sqrt(13.0) * margin) return 5;
    if (w < (2.0 + sqrt(3.0)) / 2.0 * margin) return 6;
    if (w < (sqrt(6.0) + sqrt(2.0)) / 2.0 * margin) return 7;
    return -1;
}

/* Cells along one axis of length L: explicit if m_req > 0; otherwise the
 * smallest even m with L/m < w_max when w_max > 0, else the largest even m
 * with L/m >= w_min. */
static int choose_cells(double L, int m_req, double w_min, double w_max)
{
    if (m_req > 0) return m_req;
    if (w_max > 0.0) {
        int m = 2 * (int)floor(L / (2.0 * w_max));
        while (L / (double)m >= w_max) m += 2;
        return m;
    }
    int m = 2 * (int)floor(L / (2.0 * w_min));
    while (m > 0 && L / (double)m < w_min) m -= 2;
    return m;
}

/* Box of the triangular lattice at packing fraction phi: area
 * A = N pi / (4 phi) for unit diameter, lattice constant a with
 * A = nx ny a^2 sqrt(3)/2, row spacing h = a sqrt(3)/2. */
static void lattice_box(int nx, int ny, double phi, double *a, double *h,
                        double *Lx, double *Ly)
{
    double N = (double)nx * (double)ny;
    double A = N * 3.14159265358979323846 / (4.0 * phi);
    *a = sqrt(2.0 * A / (sqrt(3.0) * N));
    *h = *a * sqrt(3.0) / 2.0;
    *Lx = (double)nx * *a;
    *Ly = (double)ny * *h;
}

int oracle_geometry(int nx, int ny, double phi, int mx_req, int my_req,
                    double w_min, double w_max, int *mx, int *my, float *wx,
                    float *wy, int *cap, double *Lx, double *Ly)
{
    if (nx < 1 || ny < 2 || (ny & 1) || !(phi > 0.0 && phi < 0.9)) return ORC_EINVAL;
    double a, h;
    lattice_box(nx, ny, phi, &a, &h, Lx, Ly);
    if (w_min <= 0.0) w_min = 1.0;
    *mx = choose_cells(*Lx, mx_req, w_min, w_max);
    *my = choose_cells(*Ly, my_req, w_min, w_max);
    if (*mx < 4 || *my < 4 || (*mx & 1) || (*my & 1)) return ORC_EGEOM;
    *wx = (float)(*Lx / (double)*mx);
    *wy = (float)(*Ly / (double)*my);
    if (!(*wx >= 1.0f && *wy >= 1.0f)) return ORC_EGEOM;
    double wmax = *wx > *wy ? (double)*wx : (double)*wy;
    *cap = capacity_for_width(wmax);
    if (*cap < 0) return ORC_EGEOM;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * System state.
 * ------------------------------------------------------------------------ */
typedef struct oracle_sys {
    int mx, my, C, cap;
    int64_t N;
    float wx, wy;
    float delta;
    int n_moves;
    uint32_t key[2];
    uint64_t sweep;
    uint64_t trials, accepts;
    int flags;      /* bit 0: displacement accumulators, bit 1: tags, bit 3: disk moves,
                       bits 4, 5: no particle / no set shuffle */
    int cell_order; /* 0 row-major, 1 reversed, 2 scrambled (order test) */
    int threads;    /* OpenMP threads over the cells of one set (default 1) */
    /* disk[c*cap + i] (Sec. 3.1), double buffer for the shift (Alg. 4) */
    float *disk_x, *disk_y, *dbl_x, *dbl_y;
    float *acc_x, *acc_y, *dacc_x, *dacc_y;
    uint32_t *tag, *dtag;
    int *n, *n_dbl;
    /* bit s of accept_bits[c]: trial s (s < 32) of the cell's latest update
     * was accepted; a sweep updates every cell once */
    uint32_t *accept_bits;
} oracle_sys;

#define FLAG_ACC 1
#define FLAG_TAG 2
#define FLAG_DISK 8 /* in-circle proposals instead of the square */
/* The two shuffles the paper switches off in its balance test (Sec. 2.4,
 * Table 1).  Without the particle shuffle detailed balance is lost; the
 * set shuffle is not needed for correct sampling.  Diagnostic only. */
#define FLAG_NO_PARTICLE_SHUFFLE 16
#define FLAG_NO_SET_SHUFFLE 32
/* The two cell-leaving pitfalls of Sec. 2.4, diagnostic only.  LEAVE: a
 * move may take the disk out of its cell; it stays in the cell's list with
 * a local coordinate outside (0, w] until the sweep's shift re-homes it.
 * LEAVE_ONCE: the same, with n_M = n for every cell update, so each disk
 * is moved exactly once per sweep.  To keep the 3x3 overlap test complete
 * and the cells of one set independent, a move is rejected if it takes
 * the disk more than e = (w - 1)/2 outside its cell (per axis): two disks
 * displaced towards each other are then still a full cell width apart
 * minus 2e >= 1.  With w = 1 the bound is 0 and LEAVE is the plain chain. */
#define FLAG_LEAVE 64
#define FLAG_LEAVE_ONCE 128
#define FLAG_LEAVE_ANY (FLAG_LEAVE | FLAG_LEAVE_ONCE)

static void *xcalloc(size_t n, size_t sz)
{
    void *p = calloc(n ? n : 1, sz);
    if (!p) abort();
    return p;
}

static oracle_sys *alloc_sys(int mx, int my, float wx, float wy, int cap,
                             int flags)
{
    oracle_sys *S = (oracle_sys *)xcalloc(1, sizeof(oracle_sys));
    S->mx = mx; S->my = my; S->C = mx * my; S->cap = cap;
    S->wx = wx; S->wy = wy; S->flags = flags;
    S->threads = 1;
    size_t slots = (size_t)S->C * (size_t)cap;
    S->disk_x = (float *)xcalloc(slots, sizeof(float));
    S->disk_y = (float *)xcalloc(slots, sizeof(float));
    S->dbl_x = (float *)xcalloc(slots, sizeof(float));
    S->dbl_y = (float *)xcalloc(slots, sizeof(float));
    S->acc_x = (float *)xcalloc(slots, sizeof(float));
    S->acc_y = (float *)xcalloc(slots, sizeof(float));
    S->dacc_x = (float *)xcalloc(slots, sizeof(float));
    S->dacc_y = (float *)xcalloc(slots, sizeof(float));
    S->tag = (uint32_t *)xcalloc(slots, sizeof(uint32_t));
    S->dtag = (uint32_t *)xcalloc(slots, sizeof(uint32_t));
    S->n = (int *)xcalloc((size_t)S->C, sizeof(int));
    S->n_dbl = (int *)xcalloc((size_t)S->C, sizeof(int));
    S->accept_bits = (uint32_t *)xcalloc((size_t)S->C, sizeof(uint32_t));
    return S;
}

void oracle_destroy(oracle_sys *S)
{
    if (!S) return;
    free(S->disk_x); free(S->disk_y); free(S->dbl_x); free(S->dbl_y);
    free(S->acc_x); free(S->acc_y); free(S->dacc_x); free(S->dacc_y);
    free(S->tag); free(S->dtag); free(S->n); free(S->n_dbl);
    free(S->accept_bits);
    free(S);
}

/* Initial condition: triangular lattice (nx columns, ny rows, ny even),
 * site (i,j) at x = (i + 1/4 + (j odd)/2) a, y = (j + 1/2) h, computed in
 * FP64; the +1/4 keeps sites off the cell edges.  A disk goes to cell
 * cx = ceil(x/wx) - 1 (so x lies in (cx wx, (cx+1) wx]) with local
 * coordinate (float)(x - cx wx); within a cell, particles are listed in
 * ascending lattice index j*nx + i. */
oracle_sys *oracle_create(int nx, int ny, double phi, int mx_req, int my_req,
                          double w_min, double w_max, float delta, int n_moves,
                          uint32_t seed, uint32_t replica, int flags, int *status)
{
    int mx, my, cap;
    float wx, wy;
    double Lx, Ly;
    int st = oracle_geometry(nx, ny, phi, mx_req, my_req, w_min, w_max, &mx, &my,
                             &wx, &wy, &cap, &Lx, &Ly);
    if (st != ORC_OK) { if (status) *status = st; return NULL; }
    if (!(delta > 0.0f) || delta > 0.5f * (wx < wy ? wx : wy) || n_moves < 0) {
        if (status) *status = ORC_EINVAL;
        return NULL;
    }
    oracle_sys *S = alloc_sys(mx, my, wx, wy, cap, flags);
    S->N = (int64_t)nx * ny;
    S->delta = delta;
    S->n_moves = n_moves;
    S->key[0] = seed; S->key[1] = replica;
    double a, h, Lx2, Ly2;
    lattice_box(nx, ny, phi, &a, &h, &Lx2, &Ly2);
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double x = ((double)i + 0.25 + 0.5 * (double)(j & 1)) * a;
            double y = ((double)j + 0.5) * h;
            int cx = (int)ceil(x / (double)wx) - 1;
            int cy = (int)ceil(y / (double)wy) - 1;
            if (cx < 0 || cx >= mx || cy < 0 || cy >= my) {
                oracle_destroy(S);
                if (status) *status = ORC_EGEOM;
                return NULL;
            }
            float lx = (float)(x - (double)cx * (double)wx);
            float ly = (float)(y - (double)cy * (double)wy);
            int c = cy * mx + cx;
            if (S->n[c] >= cap || !(lx > 0.0f && lx <= wx && ly > 0.0f && ly <= wy)) {
                oracle_destroy(S);
                if (status) *status = ORC_EGEOM;
                return NULL;
            }
            int slot = c * cap + S->n[c];
            S->disk_x[slot] = lx;
            S->disk_y[slot] = ly;
            S->tag[slot] = (uint32_t)(j * nx + i);
            S->n[c] += 1;
        }
    }
    if (status) *status = ORC_OK;
    return S;
}

/* An empty system of the given grid, to be filled with oracle_set_state. */
oracle_sys *oracle_create_grid(int mx, int my, float wx, float wy, float delta,
                               int n_moves, uint32_t seed, uint32_t replica,
                               int flags, int *status)
{
    if (mx < 4 || my < 4 || (mx & 1) || (my & 1) || !(wx >= 1.0f && wy >= 1.0f)) {
        if (status) *status = ORC_EGEOM;
        return NULL;
    }
    int cap = capacity_for_width(wx > wy ? (double)wx : (double)wy);
    if (cap < 0) { if (status) *status = ORC_EGEOM; return NULL; }
    if (!(delta > 0.0f) || delta > 0.5f * (wx < wy ? wx : wy) || n_moves < 0) {
        if (status) *status = ORC_EINVAL;
        return NULL;
    }
    oracle_sys *S = alloc_sys(mx, my, wx, wy, cap, flags);
    S->delta = delta; S->n_moves = n_moves;
    S->key[0] = seed; S->key[1] = replica;
    if (status) *status = ORC_OK;
    return S;
}

void oracle_info(const oracle_sys *S, int *mx, int *my, float *wx, float *wy,
                 int *cap, int64_t *N)
{
    *mx = S->mx; *my = S->my; *wx = S->wx; *wy = S->wy; *cap = S->cap; *N = S->N;
}

void oracle_set_delta(oracle_sys *S, float delta) { S->delta = delta; }
float oracle_get_delta(const oracle_sys *S) { return S->delta; }
void oracle_set_seed(oracle_sys *S, uint32_t seed) { S->key[0] = seed; }
void oracle_set_n_moves(oracle_sys *S, int n_moves) { S->n_moves = n_moves; }
void oracle_set_cell_order(oracle_sys *S, int mode) { S->cell_order = mode; }
uint64_t oracle_get_sweep(const oracle_sys *S) { return S->sweep; }

void oracle_get_counters(const oracle_sys *S, uint64_t *trials, uint64_t *accepts)
{
    *trials = S->trials;
    *accepts = S->accepts;
}

/* ------------------------------------------------------------------------
 * One cell update (Alg. 1, Alg. 2).
 * ------------------------------------------------------------------------ */
static int wrap(int i, int m) { return (i % m + m) % m; }

static void swap_slots(oracle_sys *S, int a, int b)
{
    float t;
    uint32_t u;
    t = S->disk_x[a]; S->disk_x[a] = S->disk_x[b]; S->disk_x[b] = t;
    t = S->disk_y[a]; S->disk_y[a] = S->disk_y[b]; S->disk_y[b] = t;
    t = S->acc_x[a]; S->acc_x[a] = S->acc_x[b]; S->acc_x[b] = t;
    t = S->acc_y[a]; S->acc_y[a] = S->acc_y[b]; S->acc_y[b] = t;
    u = S->tag[a]; S->tag[a] = S->tag[b]; S->tag[b] = u;
}

/* Does a disk at (xm, ym) in cell (cx, cy)'s frame overlap any disk of the
 * 3x3 neighbourhood other than slot `self` of the cell itself?  A neighbour
 * at offset (ox, oy) is seen at (x + ox*wx, y + oy*wy); the translation is
 * one of -w, 0, +w exactly (Sec. 3.1).  Overlap iff r^2 < sigma^2 = 1
 * (Alg. 2); touching disks are allowed.  The paper fixes no rounding for
 * r^2; the chain takes ddx*ddx rounded, plus ddy*ddy by one fused
 * multiply-add (fmaf rounds once). */
static int overlaps(const oracle_sys *S, int cx, int cy, int self, float xm, float ym)
{
    for (int oy = -1; oy <= 1; ++oy) {
        int ny_ = wrap(cy + oy, S->my);
        float ty = oy < 0 ? -S->wy : (oy > 0 ? S->wy : 0.0f);
        for (int ox = -1; ox <= 1; ++ox) {
            int nx_ = wrap(cx + ox, S->mx);
            float tx = ox < 0 ? -S->wx : (ox > 0 ? S->wx : 0.0f);
            int nc = ny_ * S->mx + nx_;
            int own = (ox == 0 && oy == 0);
            for (int j = 0; j < S->n[nc]; ++j) {
                int slot = nc * S->cap + j;
                if (own && slot == self) continue;
                float px = S->disk_x[slot] + tx;
                float py = S->disk_y[slot] + ty;
                float ddx = xm - px;
                float ddy = ym - py;
                float r2 = fmaf(ddy, ddy, ddx * ddx);
                if (r2 < 1.0f) return 1;
            }
        }
    }
    return 0;
}

/* One cell update; the cell's trials and accepts are added to *trials and
 * *accepts, so that cells of one set can be updated by several threads. */
static void cell_update(oracle_sys *S, int cx, int cy, uint64_t *trials, uint64_t *accepts)
{
    int c = cy * S->mx + cx;
    int n = S->n[c];
    S->accept_bits[c] = 0;
    if (n == 0) return; /* nothing to move (Alg. 2) */
    int base = c * S->cap;
    uint32_t words[4];

    /* rng.shuffle(c.particles): Fisher-Yates (Durstenfeld) over the stored
     * list; the k-th draw (k = 0,1,...) picks the partner of position n-1-k.
     * Skipped, and the list visited in stored order, under the ablation. */
    int shuffles = (S->flags & FLAG_NO_PARTICLE_SHUFFLE) ? 0 : n - 1;
    for (int k = 0; k < shuffles; ++k) {
        if ((k & 3) == 0) stream_block((uint32_t)c, S->sweep, TAG_SHUFFLE + (uint32_t)(k >> 2), S->key, words);
        int i = n - 1 - k;
        int j = (int)oracle_bounded(words[k & 3], (uint32_t)(i + 1));
        swap_slots(S, base + i, base + j);
    }

    /* n_M trial moves, particle list[s mod n] (Alg. 1); under the
     * leave-once pitfall n of them, one per disk.  The window a trial
     * position must stay in: the cell, or under the leaving pitfalls the
     * cell grown by e = (w - 1)/2 per axis. */
    int leave = (S->flags & FLAG_LEAVE_ANY) != 0;
    int trials_here = (S->flags & FLAG_LEAVE_ONCE) ? n : S->n_moves;
    float ex = leave ? (S->wx - 1.0f) * 0.5f : 0.0f;
    float ey = leave ? (S->wy - 1.0f) * 0.5f : 0.0f;
    float lox = -ex, hix = S->wx + ex, loy = -ey, hiy = S->wy + ey;
    for (int s = 0; s < trials_here; ++s) {
        if ((s & 3) == 0) stream_block((uint32_t)c, S->sweep, TAG_TRIAL + (uint32_t)(s >> 2), S->key, words);
        int slot = base + visit_slot(s, n);
        float dx, dy;
        if (S->flags & FLAG_DISK)
            oracle_disk_displacement(words[s & 3], S->delta, &dx, &dy);
        else
            oracle_trial_displacement(words[s & 3], S->delta, &dx, &dy);
        float xm = S->disk_x[slot] + dx;
        float ym = S->disk_y[slot] + dy;
        int in_cell = xm > lox && xm <= hix && ym > loy && ym <= hiy;
        *trials += 1;
        if (in_cell && !overlaps(S, cx, cy, slot, xm, ym)) {
            S->disk_x[slot] = xm;
            S->disk_y[slot] = ym;
            if (S->flags & FLAG_ACC) {
                S->acc_x[slot] = S->acc_x[slot] + dx;
                S->acc_y[slot] = S->acc_y[slot] + dy;
            }
            *accepts += 1;
            if (s < 32) S->accept_bits[c] |= 1u << s;
        }
    }
}

/* The accept bits of every cell (C entries, row-major cells). */
void oracle_get_accept_log(const oracle_sys *S, uint32_t *out)
{
    memcpy(out, S->accept_bits, sizeof(uint32_t) * (size_t)S->C);
}

/* Sub-sweep over checkerboard set Q (Eq. 1): cells with (cx mod 2) + 2 (cy
 * mod 2) == Q, i.e. 0=a, 1=b, 2=c, 3=d.  Cells of one set never interact
 * (w >= sigma), so the visiting order cannot change the result; the order
 * mode exists to test exactly that. */
void oracle_subsweep(oracle_sys *S, int Q)
{
    int qx = Q & 1, qy = (Q >> 1) & 1;
    int hx = S->mx / 2, hy = S->my / 2;
    int count = hx * hy;
    uint64_t trials = 0, accepts = 0;
    /* Several threads only split the (independent) cells of the set among
     * them; each cell's update is the serial one. */
#ifdef _OPENMP
#pragma omp parallel for num_threads(S->threads) schedule(static) reduction(+ : trials, accepts) if (S->threads > 1)
#endif
    for (int k = 0; k < count; ++k) {
        int idx = k;
        if (S->cell_order == 1) idx = count - 1 - k;
        else if (S->cell_order == 2) idx = (int)(((int64_t)k * 7919 + 13) % count);
        int ix = idx % hx, iy = idx / hx;
        cell_update(S, 2 * ix + qx, 2 * iy + qy, &trials, &accepts);
    }
    S->trials += trials;
    S->accepts += accepts;
}

/* Threads used by every later sub-sweep (1 = serial; without OpenMP the
 * library is serial whatever is asked).  Returns the number in effect. */
int oracle_set_threads(oracle_sys *S, int threads)
{
#ifdef _OPENMP
    S->threads = threads < 1 ? 1 : threads;
#else
    (void)threads;
    S->threads = 1;
#endif
    return S->threads;
}

/* ------------------------------------------------------------------------
 * Cell shift (Alg. 4): all particles move by -f*d, i.e. the grid moves by
 * +f*d.  For f = +x the shifted coordinate is t = x - d, for f = -x it is
 * t = x + d (one FP32 operation), likewise for y.  A particle stays iff t
 * lies in (0, w]; otherwise it belongs to the neighbour cell opposite to f
 * and its coordinate there is t + w (f = +x) or t - w (f = -x).  New cell c
 * receives its own stayers in list order, then the leavers of the cell in
 * direction f in list order.  f: 0 = +x, 1 = -x, 2 = +y, 3 = -y.
 * ------------------------------------------------------------------------ */
static float shifted(float v, int f, float d)
{
    return (f == 0 || f == 2) ? v - d : v + d;
}

/* The shift under the leaving pitfalls: disks may sit up to (w - 1)/2
 * outside their cell on either axis.  Each disk's coordinates are the
 * shifted one (one FP32 operation, as above) and the other one; per axis a
 * value <= 0 sends the disk one cell down (coordinate + w), a value > w one
 * cell up (coordinate - w), one rounding each.  New cell c lists the disks
 * that land in it: first its own stayers, then the arrivals from the eight
 * neighbours in row-major order of the offset (dy, then dx), each source in
 * list order.  Without excursions only the neighbour in direction f has
 * arrivals, and this is the order above. */
static void land(float t, float w, int *off, float *u)
{
    if (t <= 0.0f) { *off = -1; *u = t + w; }
    else if (t > w) { *off = 1; *u = t - w; }
    else { *off = 0; *u = t; }
}

static void shift_cells_general(oracle_sys *S, int f, float d)
{
    int along_x = (f < 2);
    for (int cy = 0; cy < S->my; ++cy) {
        for (int cx = 0; cx < S->mx; ++cx) {
            int c = cy * S->mx + cx;
            int out = c * S->cap;
            int n_new = 0;
            for (int k = 0; k < 9; ++k) {
                /* k = 0: the cell itself; then (dy, dx) row-major without (0, 0) */
                int q = k == 0 ? 4 : (k <= 4 ? k - 1 : k);
                int ox = q % 3 - 1, oy = q / 3 - 1;
                int sx = wrap(cx + ox, S->mx), sy = wrap(cy + oy, S->my);
                int sc = sy * S->mx + sx;
                for (int i = 0; i < S->n[sc]; ++i) {
                    int slot = sc * S->cap + i;
                    float vx = S->disk_x[slot], vy = S->disk_y[slot];
                    float tx = along_x ? shifted(vx, f, d) : vx;
                    float ty = along_x ? vy : shifted(vy, f, d);
                    int mxo, myo;
                    float ux, uy;
                    land(tx, S->wx, &mxo, &ux);
                    land(ty, S->wy, &myo, &uy);
                    if (mxo != -ox || myo != -oy) continue; /* lands elsewhere */
                    if (n_new >= S->cap) { S->n_dbl[c] = -1; goto next_cell; }
                    int o = out + n_new++;
                    S->dbl_x[o] = ux;
                    S->dbl_y[o] = uy;
                    S->dacc_x[o] = S->acc_x[slot]; S->dacc_y[o] = S->acc_y[slot];
                    S->dtag[o] = S->tag[slot];
                }
            }
            S->n_dbl[c] = n_new;
        next_cell:;
        }
    }
}

void oracle_shift_cells(oracle_sys *S, int f, float d)
{
    if (S->flags & FLAG_LEAVE_ANY) {
        shift_cells_general(S, f, d);
        goto swap;
    }
    int along_x = (f < 2);
    int sgn = (f == 0 || f == 2) ? +1 : -1; /* direction of f along its axis */
    float w = along_x ? S->wx : S->wy;
    for (int cy = 0; cy < S->my; ++cy) {
        for (int cx = 0; cx < S->mx; ++cx) {
            int c = cy * S->mx + cx;
            int out = c * S->cap;
            int n_new = 0;
            /* stayers of the cell itself */
            for (int i = 0; i < S->n[c]; ++i) {
                int slot = c * S->cap + i;
                float v = along_x ? S->disk_x[slot] : S->disk_y[slot];
                float t = shifted(v, f, d);
                if (t > 0.0f && t <= w) {
                    if (n_new >= S->cap) { S->n_dbl[c] = -1; goto next_cell; }
                    int o = out + n_new++;
                    S->dbl_x[o] = along_x ? t : S->disk_x[slot];
                    S->dbl_y[o] = along_x ? S->disk_y[slot] : t;
                    S->dacc_x[o] = S->acc_x[slot]; S->dacc_y[o] = S->acc_y[slot];
                    S->dtag[o] = S->tag[slot];
                }
            }
            /* leavers of the neighbour in direction f enter this cell */
            {
                int ncx = along_x ? wrap(cx + sgn, S->mx) : cx;
                int ncy = along_x ? cy : wrap(cy + sgn, S->my);
                int nc = ncy * S->mx + ncx;
                float s = sgn > 0 ? w : -w; /* vector pointing to the neighbour */
                for (int i = 0; i < S->n[nc]; ++i) {
                    int slot = nc * S->cap + i;
                    float v = along_x ? S->disk_x[slot] : S->disk_y[slot];
                    float t = shifted(v, f, d);
                    if (t > 0.0f && t <= w) continue; /* stays in the neighbour */
                    if (n_new >= S->cap) { S->n_dbl[c] = -1; goto next_cell; }
                    int o = out + n_new++;
                    float tt = t + s;
                    S->dbl_x[o] = along_x ? tt : S->disk_x[slot];
                    S->dbl_y[o] = along_x ? S->disk_y[slot] : tt;
                    S->dacc_x[o] = S->acc_x[slot]; S->dacc_y[o] = S->acc_y[slot];
                    S->dtag[o] = S->tag[slot];
                }
            }
            S->n_dbl[c] = n_new;
        next_cell:;
        }
    }
swap:;
    /* swap the double buffers */
    float *tp;
    uint32_t *tu;
    int *ti;
    tp = S->disk_x; S->disk_x = S->dbl_x; S->dbl_x = tp;
    tp = S->disk_y; S->disk_y = S->dbl_y; S->dbl_y = tp;
    tp = S->acc_x; S->acc_x = S->dacc_x; S->dacc_x = tp;
    tp = S->acc_y; S->acc_y = S->dacc_y; S->dacc_y = tp;
    tu = S->tag; S->tag = S->dtag; S->dtag = tu;
    ti = S->n; S->n = S->n_dbl; S->n_dbl = ti;
}

/* ------------------------------------------------------------------------
 * One sweep (Alg. 1).  The sweep-global Philox block G = philox(0xFFFFFFFF,
 * sweep, TAG_SWEEP): G[0..2] shuffle the set order (Fisher-Yates on
 * [a,b,c,d]), the top two bits of G[3] choose f, its low 24 bits give
 * d = u * (w_f / 2) with u in [0,1).
 * ------------------------------------------------------------------------ */
void oracle_sweep_draws(const oracle_sys *S, uint64_t sweep, int order[4], int *f, float *d)
{
    uint32_t G[4];
    stream_block(CELL_GLOBAL, sweep, TAG_SWEEP, S->key, G);
    for (int i = 0; i < 4; ++i) order[i] = i;
    /* the set-order shuffle, skipped under the ablation (a, b, c, d always);
     * f and d come from G[3] either way */
    for (int i = 3; i >= 1 && !(S->flags & FLAG_NO_SET_SHUFFLE); --i) {
        int j = (int)oracle_bounded(G[3 - i], (uint32_t)(i + 1));
        int t = order[i]; order[i] = order[j]; order[j] = t;
    }
    *f = (int)(G[3] >> 30);
    float w = (*f < 2) ? S->wx : S->wy;
    float u = (float)(G[3] & 0xFFFFFFu) * 0x1p-24f;
    *d = u * (0.5f * w);
}

int oracle_check_capacity(const oracle_sys *S)
{
    for (int c = 0; c < S->C; ++c)
        if (S->n[c] < 0 || S->n[c] > S->cap) return ORC_ESTATE;
    return ORC_OK;
}

int oracle_sweep(oracle_sys *S, int64_t n_sweeps)
{
    for (int64_t k = 0; k < n_sweeps; ++k) {
        int order[4], f;
        float d;
        oracle_sweep_draws(S, S->sweep, order, &f, &d);
        for (int i = 0; i < 4; ++i) oracle_subsweep(S, order[i]);
        oracle_shift_cells(S, f, d);
        if (oracle_check_capacity(S) != ORC_OK) return ORC_ESTATE;
        S->sweep += 1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * State exchange in compressed-row form: cells in row-major order, each
 * cell's particles in list order; xy interleaved (x0,y0,x1,y1,...),
 * start[C+1] offsets.
 * ------------------------------------------------------------------------ */
int64_t oracle_num_particles(const oracle_sys *S)
{
    int64_t total = 0;
    for (int c = 0; c < S->C; ++c) total += S->n[c];
    return total;
}

void oracle_get_state(const oracle_sys *S, float *xy, uint32_t *start, uint64_t *sweep)
{
    uint32_t off = 0;
    for (int c = 0; c < S->C; ++c) {
        start[c] = off;
        for (int i = 0; i < S->n[c]; ++i) {
            int slot = c * S->cap + i;
            xy[2 * (size_t)off] = S->disk_x[slot];
            xy[2 * (size_t)off + 1] = S->disk_y[slot];
            ++off;
        }
    }
    start[S->C] = off;
    if (sweep) *sweep = S->sweep;
}

void oracle_get_aux(const oracle_sys *S, float *acc, uint32_t *tag)
{
    size_t off = 0;
    for (int c = 0; c < S->C; ++c) {
        for (int i = 0; i < S->n[c]; ++i) {
            int slot = c * S->cap + i;
            if (acc) { acc[2 * off] = S->acc_x[slot]; acc[2 * off + 1] = S->acc_y[slot]; }
            if (tag) tag[off] = S->tag[slot];
            ++off;
        }
    }
}

void oracle_reset_acc(oracle_sys *S)
{
    size_t slots = (size_t)S->C * (size_t)S->cap;
    memset(S->acc_x, 0, slots * sizeof(float));
    memset(S->acc_y, 0, slots * sizeof(float));
}

/* Load a state; tags are optional (NULL -> 0,1,2,... in list order). */
int oracle_set_state(oracle_sys *S, const float *xy, const uint32_t *start,
                     uint64_t sweep, const uint32_t *tag)
{
    if (start[0] != 0) return ORC_ESTATE;
    for (int c = 0; c < S->C; ++c) {
        if (start[c + 1] < start[c]) return ORC_ESTATE;
        uint32_t cnt = start[c + 1] - start[c];
        if (cnt > (uint32_t)S->cap) return ORC_ESTATE;
        for (uint32_t k = start[c]; k < start[c + 1]; ++k) {
            float x = xy[2 * (size_t)k], y = xy[2 * (size_t)k + 1];
            if (!(x > 0.0f && x <= S->wx && y > 0.0f && y <= S->wy)) return ORC_ESTATE;
        }
    }
    for (int c = 0; c < S->C; ++c) {
        S->n[c] = (int)(start[c + 1] - start[c]);
        for (int i = 0; i < S->n[c]; ++i) {
            size_t k = start[c] + (size_t)i;
            int slot = c * S->cap + i;
            S->disk_x[slot] = xy[2 * k];
            S->disk_y[slot] = xy[2 * k + 1];
            S->acc_x[slot] = 0.0f; S->acc_y[slot] = 0.0f;
            S->tag[slot] = tag ? tag[k] : (uint32_t)k;
        }
    }
    S->N = start[S->C];
    S->sweep = sweep;
    S->trials = S->accepts = 0; /* counters run from the loaded state */
    return ORC_OK;
}

/* Smallest r^2 over ordered pairs (k, j != k) of the 3x3 neighbourhoods,
 * evaluated in k's frame as in the trial moves (2.0 if there is no pair). */
float oracle_min_pair_r2(const oracle_sys *S)
{
    float best = 2.0f;
    for (int cy = 0; cy < S->my; ++cy)
        for (int cx = 0; cx < S->mx; ++cx) {
            int c = cy * S->mx + cx;
            for (int i = 0; i < S->n[c]; ++i) {
                int self = c * S->cap + i;
                float xk = S->disk_x[self], yk = S->disk_y[self];
                for (int oy = -1; oy <= 1; ++oy) {
                    int ncy = wrap(cy + oy, S->my);
                    float ty = oy < 0 ? -S->wy : (oy > 0 ? S->wy : 0.0f);
                    for (int ox = -1; ox <= 1; ++ox) {
                        int ncx = wrap(cx + ox, S->mx);
                        float tx = ox < 0 ? -S->wx : (ox > 0 ? S->wx : 0.0f);
                        int nc = ncy * S->mx + ncx;
                        for (int j = 0; j < S->n[nc]; ++j) {
                            int slot = nc * S->cap + j;
                            if (slot == self) continue;
                            float ddx = xk - (S->disk_x[slot] + tx);
                            float ddy = yk - (S->disk_y[slot] + ty);
                            float r2 = ddx * ddx + ddy * ddy;
                            if (r2 < best) best = r2;
                        }
                    }
                }
            }
        }
    return best;
}

/* Invariant check: ordered pairs (k, j) with r^2 < 1 - 2^-20 evaluated in
 * k's frame as in the trial moves.  Every accepted move has r^2 >= 1 in the
 * mover's frame with the coordinates of that moment.  The pair can read
 * lower later for two reasons, both rounding: (i) in the partner's frame the
 * translation by w and the differences round differently (a few ulp of
 * r^2 ~ 1, i.e. below 2^-21); (ii) each rebin re-expresses a coordinate in
 * the new frame with one rounding of at most half an ulp of a value below 2
 * (2^-24 absolute), so r moves by at most 2^-23 per rebin while neither disk
 * of the pair moves.  1 - 2^-20 (about 9.5e-7) covers (i) plus a few tens of
 * rebins of (ii); the tests also record the smallest r^2 reached. */
int64_t oracle_count_overlaps(const oracle_sys *S)
{
    const float r2min = 1.0f - 0x1p-20f;
    int64_t bad = 0;
    for (int cy = 0; cy < S->my; ++cy)
        for (int cx = 0; cx < S->mx; ++cx) {
            int c = cy * S->mx + cx;
            for (int i = 0; i < S->n[c]; ++i) {
                int self = c * S->cap + i;
                float xk = S->disk_x[self], yk = S->disk_y[self];
                for (int oy = -1; oy <= 1; ++oy) {
                    int ncy = wrap(cy + oy, S->my);
                    float ty = oy < 0 ? -S->wy : (oy > 0 ? S->wy : 0.0f);
                    for (int ox = -1; ox <= 1; ++ox) {
                        int ncx = wrap(cx + ox, S->mx);
                        float tx = ox < 0 ? -S->wx : (ox > 0 ? S->wx : 0.0f);
                        int nc = ncy * S->mx + ncx;
                        for (int j = 0; j < S->n[nc]; ++j) {
                            int slot = nc * S->cap + j;
                            if (slot == self) continue;
                            float ddx = xk - (S->disk_x[slot] + tx);
                            float ddy = yk - (S->disk_y[slot] + ty);
                            bad += (ddx * ddx + ddy * ddy < r2min);
                        }
                    }
                }
            }
        }
    return bad;
}

/* ------------------------------------------------------------------------
 * Pair histogram for the contact value of g(r) (Sec. 4, Eqs. gR and R):
 * ordered pairs (k, j != k) with r in [1, 1 + 200*1e-4), bin b iff
 * E_b <= r^2 < E_{b+1}, E_b = (float)((1 + b*1e-4)^2) from FP64.  r^2 is
 * evaluated in k's frame exactly as in the overlap test.  When a cell is
 * narrower than the histogram range the scan reaches two cells out.
 * ------------------------------------------------------------------------ */
void oracle_hist_edges(float edges[HIST_BINS + 1])
{
    for (int b = 0; b <= HIST_BINS; ++b) {
        double r = 1.0 + (double)b * 1e-4;
        edges[b] = (float)(r * r);
    }
}

int oracle_pair_histogram(const oracle_sys *S, uint64_t hist[HIST_BINS])
{
    float E[HIST_BINS + 1];
    oracle_hist_edges(E);
    double rmax = 1.0 + HIST_BINS * 1e-4;
    int Rx = ((double)S->wx >= rmax) ? 1 : 2;
    int Ry = ((double)S->wy >= rmax) ? 1 : 2;
    /* the reach must not wrap onto the same cell twice */
    if (S->mx < 2 * Rx + 2 || S->my < 2 * Ry + 2) return ORC_EGEOM;
    for (int b = 0; b < HIST_BINS; ++b) hist[b] = 0;
    for (int cy = 0; cy < S->my; ++cy)
        for (int cx = 0; cx < S->mx; ++cx) {
            int c = cy * S->mx + cx;
            for (int i = 0; i < S->n[c]; ++i) {
                int self = c * S->cap + i;
                float xk = S->disk_x[self], yk = S->disk_y[self];
                for (int oy = -Ry; oy <= Ry; ++oy) {
                    int ncy = wrap(cy + oy, S->my);
                    float ty = (float)oy * S->wy;
                    for (int ox = -Rx; ox <= Rx; ++ox) {
                        int ncx = wrap(cx + ox, S->mx);
                        float tx = (float)ox * S->wx;
                        int nc = ncy * S->mx + ncx;
                        for (int j = 0; j < S->n[nc]; ++j) {
                            int slot = nc * S->cap + j;
                            if (slot == self) continue;
                            float px = S->disk_x[slot] + tx;
                            float py = S->disk_y[slot] + ty;
                            float ddx = xk - px;
                            float ddy = yk - py;
                            float r2 = ddx * ddx + ddy * ddy;
                            if (r2 < E[0] || r2 >= E[HIST_BINS]) continue;
                            int lo = 0, hi = HIST_BINS; /* E[lo] <= r2 < E[hi] */
                            while (hi - lo > 1) {
                                int mid = (lo + hi) / 2;
                                if (r2 >= E[mid]) lo = mid; else hi = mid;
                            }
                            hist[lo] += 1;
                        }
                    }
                }
            }
        }
    return ORC_OK;
}

/* Plain acceptance-ratio tuner (equilibration only): with a = accepts /
 * trials over the last window (FP64), delta <- delta * clamp(a / 0.3, 0.5,
 * 2), clamped to [1e-3, min(wx, wy) / 2]. */
float oracle_tuned_delta(float delta, uint64_t trials, uint64_t accepts, float wx, float wy)
{
    if (trials == 0) return delta;
    double a = (double)accepts / (double)trials;
    double r = a / 0.3;
    if (r < 0.5) r = 0.5;
    if (r > 2.0) r = 2.0;
    double nd = (double)delta * r;
    double hi = 0.5 * (double)(wx < wy ? wx : wy);
    if (nd < 1e-3) nd = 1e-3;
    if (nd > hi) nd = hi;
    return (float)nd;
}
