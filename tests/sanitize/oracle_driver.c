/* Sanitizer driver (test infrastructure): runs the C oracle's chain, its
 * error paths and the 3D and serial references under
 * -fsanitize=address,undefined.  Exit status 0 iff every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_sys oracle_sys;
oracle_sys *oracle_create(int nx, int ny, double phi, int mx_req, int my_req, double w_min,
                          double w_max, float delta, int n_moves, uint32_t seed, uint32_t replica,
                          int flags, int *status);
oracle_sys *oracle_create_grid(int mx, int my, float wx, float wy, float delta, int n_moves,
                               uint32_t seed, uint32_t replica, int flags, int *status);
void oracle_destroy(oracle_sys *S);
int oracle_sweep(oracle_sys *S, int64_t n_sweeps);
void oracle_shift_cells(oracle_sys *S, int f, float d);
int64_t oracle_num_particles(const oracle_sys *S);
void oracle_get_state(const oracle_sys *S, float *xy, uint32_t *start, uint64_t *sweep);
int oracle_set_state(oracle_sys *S, const float *xy, const uint32_t *start, uint64_t sweep,
                     const uint32_t *tag);
void oracle_info(const oracle_sys *S, int *mx, int *my, float *wx, float *wy, int *cap, int64_t *N);
int64_t oracle_count_overlaps(const oracle_sys *S);
int oracle_pair_histogram(const oracle_sys *S, uint64_t hist[200]);
int oracle_set_threads(oracle_sys *S, int threads);

typedef struct sphere_sys sphere_sys;
sphere_sys *sphere_create(int nx, int ny, int nz, double eta, int mx, int my, int mz, double w_max,
                          float delta, int n_moves, uint32_t seed, uint32_t replica, int *status);
void sphere_destroy(sphere_sys *S);
int sphere_sweep(sphere_sys *S, int64_t n_sweeps);
int64_t sphere_count_overlaps(const sphere_sys *S);

typedef struct serial_sys serial_sys;
serial_sys *serial_create(int64_t N, const double *x, const double *y, double Lx, double Ly,
                          double delta, uint64_t seed);
void serial_destroy(serial_sys *S);
void serial_run(serial_sys *S, int64_t n_trials);

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);      \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main(void)
{
    int st = 0;
    /* the chain: lattice, sweeps with accumulators, tags and accept bits */
    oracle_sys *S = oracle_create(24, 24, 0.70, 0, 0, 1.0, 1.41421356, 0.15f, 4, 1, 0, 1 | 2 | 4, &st);
    CHECK(S && st == 0);
    CHECK(oracle_sweep(S, 40) == 0);
    oracle_set_threads(S, 2);
    CHECK(oracle_sweep(S, 10) == 0);
    oracle_shift_cells(S, 3, 0.3f);
    CHECK(oracle_count_overlaps(S) == 0);
    uint64_t hist[200];
    CHECK(oracle_pair_histogram(S, hist) == 0);
    int mx, my, cap;
    float wx, wy;
    int64_t N;
    oracle_info(S, &mx, &my, &wx, &wy, &cap, &N);
    float *xy = malloc(sizeof(float) * 2 * (size_t)N);
    uint32_t *start = malloc(sizeof(uint32_t) * ((size_t)mx * my + 1));
    uint64_t sw = 0;
    oracle_get_state(S, xy, start, &sw);
    CHECK(sw == 50 && start[mx * my] == (uint32_t)N);
    /* set_state: a good state, then each kind of bad one */
    oracle_sys *G = oracle_create_grid(mx, my, wx, wy, 0.15f, 4, 1, 0, 3, &st);
    CHECK(G);
    CHECK(oracle_set_state(G, xy, start, sw, NULL) == 0);
    CHECK(oracle_sweep(G, 3) == 0);
    start[1] += 1;                               /* offsets out of order somewhere */
    start[2] = start[1] + (uint32_t)cap + 1;     /* a cell above capacity */
    CHECK(oracle_set_state(G, xy, start, sw, NULL) != 0);
    oracle_get_state(S, xy, start, &sw);
    xy[0] = -1.0f;                               /* coordinate outside its cell */
    CHECK(oracle_set_state(G, xy, start, sw, NULL) != 0);
    start[0] = 1;                                /* malformed first offset */
    CHECK(oracle_set_state(G, xy, start, sw, NULL) != 0);
    CHECK(oracle_create_grid(5, 4, 1.2f, 1.2f, 0.1f, 4, 1, 0, 0, &st) == NULL && st != 0);
    CHECK(oracle_create(24, 24, 0.70, 0, 0, 1.0, 0.0, 5.0f, 4, 1, 0, 0, &st) == NULL);
    free(xy);
    free(start);
    oracle_destroy(G);
    oracle_destroy(S);
    /* in-circle proposals and the shuffle ablations */
    S = oracle_create(16, 16, 0.72, 0, 0, 1.0, 1.932, 0.1f, 9, 3, 1, 8 | 16 | 32, &st);
    CHECK(S);
    CHECK(oracle_sweep(S, 20) == 0 && oracle_count_overlaps(S) == 0);
    oracle_destroy(S);
    /* hard spheres */
    sphere_sys *P = sphere_create(8, 8, 8, 0.40, 0, 0, 0, 0.0, 0.1f, 4, 1, 0, &st);
    CHECK(P);
    CHECK(sphere_sweep(P, 10) == 0 && sphere_count_overlaps(P) == 0);
    sphere_destroy(P);
    /* serial reference */
    double x[3] = {1.0, 3.0, 5.0}, y[3] = {1.0, 3.0, 5.0};
    serial_sys *R = serial_create(3, x, y, 8.0, 8.0, 0.5, 42);
    CHECK(R);
    serial_run(R, 10000);
    serial_destroy(R);
    printf("sanitized oracle run ok\n");
    return 0;
}
