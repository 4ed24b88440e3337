/*
 * serial_ref.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain serial single-particle Metropolis for hard disks in FP64 (the
 * textbook method the paper contrasts with, Sec. 1 and the caption of
 * Fig. 1): pick a disk uniformly at random, displace it uniformly in the
 * square [-delta, delta)^2, keep the move iff it creates no overlap.  A cell
 * list of cells at least sigma wide limits the overlap check to nine cells.
 * It is a different Markov chain with the same equilibrium as the
 * checkerboard chain, so equilibrium observables of the two must agree; it
 * shares no code with the checkerboard oracle.
 *
 * Global FP64 coordinates in [0, Lx) x [0, Ly), periodic, minimum image.
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct serial_sys {
    int64_t N;
    double Lx, Ly, delta;
    int gx, gy;         /* cell grid for the neighbour search */
    double cwx, cwy;    /* cell widths (>= 1) */
    int cellcap;
    double *x, *y;
    int *cell_of;       /* cell index of each disk */
    int *slot_of;       /* slot within that cell */
    int *members;       /* members[c * cellcap + k] = disk index */
    int *count;
    uint64_t rng;
    uint64_t trials, accepts;
} serial_sys;

static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform01(serial_sys *S)
{
    return (double)(splitmix64(&S->rng) >> 11) * 0x1p-53;
}

static int cell_index(const serial_sys *S, double x, double y)
{
    int cx = (int)(x / S->cwx);
    int cy = (int)(y / S->cwy);
    if (cx >= S->gx) cx = S->gx - 1;
    if (cy >= S->gy) cy = S->gy - 1;
    return cy * S->gx + cx;
}

static void cell_insert(serial_sys *S, int64_t i, int c)
{
    int k = S->count[c]++;
    if (k >= S->cellcap) abort();
    S->members[c * S->cellcap + k] = (int)i;
    S->cell_of[i] = c;
    S->slot_of[i] = k;
}

static void cell_remove(serial_sys *S, int64_t i)
{
    int c = S->cell_of[i], k = S->slot_of[i];
    int last = --S->count[c];
    int moved = S->members[c * S->cellcap + last];
    S->members[c * S->cellcap + k] = moved;
    S->slot_of[moved] = k;
}

static double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

void serial_destroy(serial_sys *S)
{
    if (!S) return;
    free(S->x); free(S->y); free(S->cell_of); free(S->slot_of);
    free(S->members); free(S->count); free(S);
}

/* Box Lx x Ly (both >= 3), positions given in FP64 global coordinates. */
serial_sys *serial_create(int64_t N, const double *x, const double *y, double Lx,
                          double Ly, double delta, uint64_t seed)
{
    serial_sys *S = (serial_sys *)calloc(1, sizeof(serial_sys));
    S->N = N; S->Lx = Lx; S->Ly = Ly; S->delta = delta;
    S->gx = (int)floor(Lx); S->gy = (int)floor(Ly);
    if (S->gx < 3 || S->gy < 3) { free(S); return NULL; }
    S->cwx = Lx / S->gx; S->cwy = Ly / S->gy;
    S->cellcap = 16;
    S->x = (double *)malloc(sizeof(double) * (size_t)N);
    S->y = (double *)malloc(sizeof(double) * (size_t)N);
    S->cell_of = (int *)malloc(sizeof(int) * (size_t)N);
    S->slot_of = (int *)malloc(sizeof(int) * (size_t)N);
    S->members = (int *)malloc(sizeof(int) * (size_t)S->gx * S->gy * S->cellcap);
    S->count = (int *)calloc((size_t)S->gx * S->gy, sizeof(int));
    S->rng = seed;
    for (int64_t i = 0; i < N; ++i) {
        S->x[i] = fmod(fmod(x[i], Lx) + Lx, Lx);
        S->y[i] = fmod(fmod(y[i], Ly) + Ly, Ly);
        cell_insert(S, i, cell_index(S, S->x[i], S->y[i]));
    }
    return S;
}

static int overlap_at(const serial_sys *S, int64_t self, double x, double y)
{
    int cx = (int)(x / S->cwx), cy = (int)(y / S->cwy);
    if (cx >= S->gx) cx = S->gx - 1;
    if (cy >= S->gy) cy = S->gy - 1;
    for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
            int c = ((cy + oy + S->gy) % S->gy) * S->gx + (cx + ox + S->gx) % S->gx;
            for (int k = 0; k < S->count[c]; ++k) {
                int j = S->members[c * S->cellcap + k];
                if (j == self) continue;
                double dx = min_image(x - S->x[j], S->Lx);
                double dy = min_image(y - S->y[j], S->Ly);
                if (dx * dx + dy * dy < 1.0) return 1;
            }
        }
    return 0;
}

/* n_trials single-particle trial moves. */
void serial_run(serial_sys *S, int64_t n_trials)
{
    for (int64_t t = 0; t < n_trials; ++t) {
        int64_t i = (int64_t)(uniform01(S) * (double)S->N);
        if (i >= S->N) i = S->N - 1;
        double dx = (2.0 * uniform01(S) - 1.0) * S->delta;
        double dy = (2.0 * uniform01(S) - 1.0) * S->delta;
        double xn = S->x[i] + dx, yn = S->y[i] + dy;
        if (xn < 0.0) xn += S->Lx; else if (xn >= S->Lx) xn -= S->Lx;
        if (yn < 0.0) yn += S->Ly; else if (yn >= S->Ly) yn -= S->Ly;
        S->trials += 1;
        if (!overlap_at(S, i, xn, yn)) {
            cell_remove(S, i);
            S->x[i] = xn; S->y[i] = yn;
            cell_insert(S, i, cell_index(S, xn, yn));
            S->accepts += 1;
        }
    }
}

void serial_counters(const serial_sys *S, uint64_t *trials, uint64_t *accepts)
{
    *trials = S->trials; *accepts = S->accepts;
}

void serial_positions(const serial_sys *S, double *x, double *y)
{
    memcpy(x, S->x, sizeof(double) * (size_t)S->N);
    memcpy(y, S->y, sizeof(double) * (size_t)S->N);
}

/* Ordered-pair histogram of r in [1, 1 + nbins*dr), bin floor((r-1)/dr),
 * added into hist. */
void serial_pair_histogram(const serial_sys *S, int nbins, double dr, uint64_t *hist)
{
    double rmax = 1.0 + nbins * dr;
    for (int64_t i = 0; i < S->N; ++i) {
        int cx = (int)(S->x[i] / S->cwx), cy = (int)(S->y[i] / S->cwy);
        if (cx >= S->gx) cx = S->gx - 1;
        if (cy >= S->gy) cy = S->gy - 1;
        int rx = S->cwx >= rmax ? 1 : 2, ry = S->cwy >= rmax ? 1 : 2;
        /* distinct neighbour cells only: on a small grid the offsets wrap */
        int seen[25], nseen = 0;
        for (int oy = -ry; oy <= ry; ++oy)
            for (int ox = -rx; ox <= rx; ++ox) {
                int c = ((cy + oy + 2 * S->gy) % S->gy) * S->gx + (cx + ox + 2 * S->gx) % S->gx;
                int dup = 0;
                for (int q = 0; q < nseen; ++q) dup |= (seen[q] == c);
                if (dup) continue;
                seen[nseen++] = c;
                for (int k = 0; k < S->count[c]; ++k) {
                    int j = S->members[c * S->cellcap + k];
                    if (j == i) continue;
                    double dx = min_image(S->x[i] - S->x[j], S->Lx);
                    double dy = min_image(S->y[i] - S->y[j], S->Ly);
                    double r = sqrt(dx * dx + dy * dy);
                    if (r < 1.0 || r >= rmax) continue;
                    int b = (int)((r - 1.0) / dr);
                    if (b >= 0 && b < nbins) hist[b] += 1;
                }
            }
    }
}
