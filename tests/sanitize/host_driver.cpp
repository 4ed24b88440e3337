// Sanitizer driver (test infrastructure): the host-only calls of
// libmpmc (geometry, buffer sizes, argument checks, error text) under
// -fsanitize=address,undefined on the host code.  Needs no GPU: none of
// these calls touches the device.  Exit status 0 iff every check holds.
#include <cstdio>
#include <cstring>

#include "mpmc.h"
#include "mpmc_sphere.h"

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main()
{
    mpmc_params p;
    std::memset(&p, 0, sizeof p);
    p.lattice_nx = p.lattice_ny = 1024;
    p.phi = 0.70;
    p.w_min = 1.0;
    p.w_max = 1.41421356;
    p.delta = 0.1f;
    p.n_moves = 4;
    p.seed = 1;
    mpmc_geometry g;
    CHECK(mpmc_geometry_of(&p, &g) == MPMC_OK);
    CHECK(g.cells_x == 826 && g.cells_y == 714 && g.capacity == 4 && g.n_particles == 1048576);
    mpmc_buffer_sizes s;
    p.flags = MPMC_FLAG_ACC | MPMC_FLAG_TAG | MPMC_FLAG_ACCEPT_LOG;
    CHECK(mpmc_required_bytes(&p, &s) == MPMC_OK && s.pos > 0 && s.acc == s.pos && s.tag > 0);
    // a batch of uneven replicas, then the error paths
    mpmc_params rp[3];
    for (int r = 0; r < 3; ++r) {
        rp[r] = p;
        rp[r].lattice_nx = rp[r].lattice_ny = 64 + 32 * r;
        rp[r].phi = 0.65 + 0.03 * r;
        rp[r].w_max = r == 2 ? 1.932 : 0.0;
        rp[r].replica = (uint32_t)r;
    }
    CHECK(mpmc_batch_required_bytes(rp, 3, &s) == MPMC_OK);
    CHECK(mpmc_batch_required_bytes(rp, 0, &s) == MPMC_EINVAL);
    rp[1].flags ^= MPMC_FLAG_TAG;   // buffer flags must agree
    CHECK(mpmc_batch_required_bytes(rp, 3, &s) == MPMC_EINVAL);
    CHECK(std::strlen(mpmc_last_error()) > 0);
    mpmc_params bad = p;
    bad.lattice_ny = 1023;          // odd row count
    CHECK(mpmc_geometry_of(&bad, &g) != MPMC_OK);
    bad = p;
    bad.cells_x = 7;                // odd grid
    bad.cells_y = 8;
    CHECK(mpmc_geometry_of(&bad, &g) != MPMC_OK);
    bad = p;
    bad.delta = 5.0f;               // wider than half a cell
    CHECK(mpmc_required_bytes(&bad, &s) != MPMC_OK);
    bad = p;
    bad.phi = 0.95;                 // beyond close packing
    CHECK(mpmc_geometry_of(&bad, &g) != MPMC_OK);
    CHECK(mpmc_geometry_of(nullptr, &g) != MPMC_OK);
    CHECK(mpmc_sweep(nullptr, 1, 1) == MPMC_EINVAL);
    CHECK(mpmc_prepare_sweeps(nullptr, 1) == MPMC_EINVAL);
    size_t wb = 0;
    CHECK(mpmc_mlp_work_bytes(100000, &wb) == MPMC_OK && wb > 0);
    CHECK(mpmc_mlp_work_bytes(-1, &wb) == MPMC_EINVAL);
    // spheres
    mpmc_sphere_params q;
    std::memset(&q, 0, sizeof q);
    q.lattice_nx = q.lattice_ny = q.lattice_nz = 40;
    q.eta = 0.45;
    q.delta = 0.05f;
    q.n_moves = 4;
    q.seed = 1;
    mpmc_sphere_geometry sg;
    CHECK(mpmc_sphere_geometry_of(&q, &sg) == MPMC_OK && sg.n_particles == 64000);
    mpmc_sphere_buffer_sizes ss;
    CHECK(mpmc_sphere_required_bytes(&q, &ss) == MPMC_OK);
    q.eta = 0.8;
    CHECK(mpmc_sphere_geometry_of(&q, &sg) != MPMC_OK);
    std::printf("sanitized host library run ok\n");
    return 0;
}
