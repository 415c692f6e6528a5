// Drives the host-only entry points of librn (rn_version, rn_strerror,
// rn_opts_default, rn_validate, rn_footprint, and rn_create's argument
// checks) over valid and invalid problems with host memory. Built together
// with the library's sources, the host code under AddressSanitizer and UBSan,
// by tests/test_host_sanitizers.py; no call here reaches a GPU. Exit status 0
// when every status is the documented one.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../include/rn.h"

static int fails = 0;
static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "unexpected: %s\n", what);
        ++fails;
    }
}

int main()
{
    expect(rn_version() > 0, "version");
    for (int s = 1; s >= -8; --s) expect(rn_strerror(s) != nullptr && std::strlen(rn_strerror(s)) > 0, "strerror");
    rn_opts o;
    expect(rn_opts_default(&o) == RN_OK, "opts_default");
    expect(rn_opts_default(nullptr) == RN_EINVAL, "opts_default(NULL)");

    const int64_t nx = 9, ny = 7, nz = 5, n = nx * ny * nz;
    std::vector<double> g0(n, 1.0), g1(n, 0.5), g2(n, 2.0);
    rn_problem p;
    std::memset(&p, 0, sizeof(p));
    p.dim = 3; p.axis = 2; p.nx = nx; p.ny = ny; p.nz = nz;
    p.g[0] = g0.data(); p.g[1] = g1.data(); p.g[2] = g2.data();
    p.mem = RN_MEM_HOST;
    expect(rn_validate(&p, &o) == RN_OK, "valid 3D");
    expect(rn_footprint(&p, &o) > (size_t)n * 40, "footprint 3D");
    o.precision = RN_MIXED;
    expect(rn_validate(&p, &o) == RN_OK && rn_footprint(&p, &o) > 0, "valid mixed");

    // entries past the lattice edge are ignored with no-flow sides, checked when periodic
    g0[nx - 1] = -1.0;
    expect(rn_validate(&p, &o) == RN_OK, "edge entry ignored");
    p.flags = RN_PERIODIC;
    expect(rn_validate(&p, &o) == RN_EINVAL, "periodic wrap entry checked");
    p.flags = 0;
    g0[nx - 1] = 1.0;
    g1[3] = std::nan("");
    expect(rn_validate(&p, &o) == RN_EINVAL, "NaN bond");
    g1[3] = INFINITY;
    expect(rn_validate(&p, &o) == RN_EINVAL, "Inf bond");
    g1[3] = -0.5;
    expect(rn_validate(&p, &o) == RN_EINVAL, "negative bond");
    g1[3] = 0.0;
    expect(rn_validate(&p, &o) == RN_OK, "removed bond");

    rn_problem q = p;
    q.dim = 4;
    expect(rn_validate(&q, &o) == RN_EINVAL && rn_footprint(&q, &o) == 0, "dim 4");
    q = p; q.axis = 3;
    expect(rn_validate(&q, &o) == RN_EINVAL, "axis 3");
    q = p; q.nz = 1;
    expect(rn_validate(&q, &o) == RN_EINVAL, "flow axis of extent 1");
    q = p; q.g[1] = nullptr;
    expect(rn_validate(&q, &o) == RN_EINVAL, "missing bond array");
    q = p; q.flags = 8;
    expect(rn_validate(&q, &o) == RN_EINVAL, "unknown flag");
    q = p; q.mem = 7;
    expect(rn_validate(&q, &o) == RN_EINVAL, "unknown memory space");
    q = p; q.nx = (int64_t)1 << 40;
    expect(rn_validate(&q, &o) == RN_EINVAL, "too many nodes");
    q = p; q.dim = 2; q.nz = 5; q.axis = 0;
    expect(rn_validate(&q, &o) == RN_EINVAL, "2D with nz > 1");
    rn_opts bad = o;
    bad.tol = 0.0;
    expect(rn_validate(&p, &bad) == RN_EINVAL, "tol 0");
    bad = o; bad.precision = 5;
    expect(rn_validate(&p, &bad) == RN_EINVAL, "precision 5");
    bad = o; bad.flags = 4;
    expect(rn_validate(&p, &bad) == RN_EINVAL, "unknown option flag");
    bad = o; bad.flags = RN_OPT_BACKBONE;
    expect(rn_validate(&p, &bad) == RN_OK && rn_footprint(&p, &bad) > rn_footprint(&p, &o), "backbone option");
    expect(rn_validate(nullptr, &o) == RN_EINVAL, "NULL problem");
    expect(rn_create(0, 0, nullptr) == RN_EINVAL, "create without an output pointer");

    // 2D, periodic across y
    const int64_t mx = 11, my = 6, m = mx * my;
    std::vector<double> h0(m, 1.0), h1(m, 1.0);
    rn_problem r;
    std::memset(&r, 0, sizeof(r));
    r.dim = 2; r.axis = 0; r.nx = mx; r.ny = my; r.nz = 1;
    r.g[0] = h0.data(); r.g[1] = h1.data();
    r.mem = RN_MEM_HOST; r.flags = RN_PERIODIC;
    expect(rn_validate(&r, &o) == RN_OK, "valid 2D periodic");
    h1[(my - 1) * mx + 3] = -1.0;   // the wrap bond of column 3
    expect(rn_validate(&r, &o) == RN_EINVAL, "2D wrap bond checked");

    std::printf("%d failures\n", fails);
    return fails != 0;
}
