// Host setup (assembly, node order, sensor location, padded rows, dt check) driven
// from a mesh file, for a build with AddressSanitizer and UndefinedBehaviorSanitizer.
// File: int32 N, E, n_obs, has_c, sensor_mode (0 node ids, 1 points), absorbing,
// n_steps; float64 dt; coords [N][3] f64; tets [E][4] i32; c [E] f64 if has_c;
// sensors (n_obs i32 node ids, or [n_obs][3] f64 points).
// Prints the pat_status and message; exit 0 on PAT_OK, 1 on an error status.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <string>
#include "pat_internal.h"
using namespace pat;
int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[7];
    double dt;
    if (fread(hdr, 4, 7, f) != 7 || fread(&dt, 8, 1, f) != 1) return 3;
    const int32_t N = hdr[0], E = hdr[1], nobs = hdr[2], has_c = hdr[3], mode = hdr[4], absorbing = hdr[5], nsteps = hdr[6];
    std::vector<double> X(size_t(N) * 3), C(has_c ? E : 0), SP(mode ? size_t(nobs) * 3 : 0);
    std::vector<int32_t> T(size_t(E) * 4), SN(mode ? 0 : nobs);
    if (fread(X.data(), 8, X.size(), f) != X.size() || fread(T.data(), 4, T.size(), f) != T.size()) return 4;
    if (has_c && fread(C.data(), 8, C.size(), f) != C.size()) return 5;
    if (mode ? fread(SP.data(), 8, SP.size(), f) != SP.size() : fread(SN.data(), 4, SN.size(), f) != SN.size()) return 6;
    fclose(f);
    pat_problem_desc d{};
    d.n_nodes = N; d.coords = X.data(); d.n_tets = E; d.tets = T.data(); d.c_tet = has_c ? C.data() : nullptr;
    d.absorbing = absorbing; d.n_obs = nobs; d.sensor_nodes = mode ? nullptr : SN.data();
    d.sensor_pos = mode ? SP.data() : nullptr; d.dt = dt; d.n_steps = nsteps; d.device = -1; d.check_dt = 1;
    HostProblem hp;
    std::string err;
    pat_status st = build_host_problem(d, hp, err);
    printf("%s: status %d %s; n %d\n", argv[1], int(st), err.c_str(), hp.n);
    return st == PAT_OK ? 0 : 1;
}
