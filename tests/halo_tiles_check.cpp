// Checks the halo tiles of the float32 step kernels (pat::build_halo_tiles) against
// their definition, on a mesh read from a binary file written by test_halo_tiles.py:
// the tiles cut the rows into consecutive runs, each tile's halo lists exactly the
// distinct rows its slots refer to, every slot's local index names its column, and
// the metadata words carry the row operands of the padded layout.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pat_internal.h"

static int fail(const std::string &m) {
    std::printf("FAIL %s\n", m.c_str());
    return 1;
}

static uint32_t fbits(double v) {
    const float f = float(v);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

int main(int argc, char **argv) {
    if (argc < 2) return fail("usage: halo_tiles_check mesh.bin");
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return fail("cannot open mesh");
    int32_t N = 0, nobs = 0, nsteps = 0;
    int64_t E = 0;
    double dt = 0;
    bool ok = std::fread(&N, 4, 1, f) == 1 && std::fread(&E, 8, 1, f) == 1;
    std::vector<double> coords(size_t(N) * 3);
    std::vector<int32_t> tets(size_t(E) * 4);
    std::vector<double> c(static_cast<size_t>(E));
    ok = ok && std::fread(coords.data(), 8, coords.size(), f) == coords.size();
    ok = ok && std::fread(tets.data(), 4, tets.size(), f) == tets.size();
    ok = ok && std::fread(c.data(), 8, c.size(), f) == c.size();
    ok = ok && std::fread(&nobs, 4, 1, f) == 1;
    std::vector<double> sp(size_t(nobs) * 3);
    ok = ok && std::fread(sp.data(), 8, sp.size(), f) == sp.size();
    ok = ok && std::fread(&dt, 8, 1, f) == 1 && std::fread(&nsteps, 4, 1, f) == 1;
    std::fclose(f);
    if (!ok) return fail("short mesh file");
    pat_problem_desc d{};
    d.n_nodes = N; d.coords = coords.data(); d.n_tets = E; d.tets = tets.data(); d.c_tet = c.data();
    d.absorbing = 1; d.n_obs = nobs; d.sensor_pos = sp.data(); d.dt = dt; d.n_steps = nsteps;
    d.device = -1; d.check_dt = 0;
    pat::HostProblem hp;
    std::string err;
    if (pat::build_host_problem(d, hp, err) != PAT_OK) return fail("setup: " + err);
    pat::HaloTiles ht;
    pat::build_halo_tiles(hp, ht);
    const int W = pat::HostProblem::kEll;
    if (int64_t(ht.desc.size()) != int64_t(ht.n_tiles) * 4) return fail("descriptor count");
    int32_t next_row = 0, next_h = 0;
    int64_t next_m = 0;
    int full = 0;
    for (int32_t t = 0; t < ht.n_tiles; ++t) {
        const int32_t *D = &ht.desc[size_t(t) * 4];
        const int32_t r0 = D[0], h0 = D[1], moff = D[2], fl = D[3];
        constexpr int FB = pat::HaloTiles::kNrBits, FM = (1 << FB) - 1;
        const int32_t nr = fl & FM, nk4 = (fl >> FB) & 255, nb4 = (fl >> (FB + 8)) & 255, nbr = (fl >> (FB + 16)) & FM;
        const std::string at = "tile " + std::to_string(t);
        if (r0 != next_row || nr < 1 || nr > pat::HaloTiles::kRows) return fail(at + ": rows");
        if (h0 != next_h || moff != next_m / 16) return fail(at + ": offsets");
        if (nk4 % 4 || nb4 % 4 || nk4 + nb4 > pat::HaloTiles::kMax) return fail(at + ": halo size");
        full += nr == pat::HaloTiles::kRows;
        // the halo lists: sorted distinct columns, padded to a multiple of 4 with the last one
        std::vector<int32_t> kc, bc;
        int32_t bnd = 0;
        for (int32_t i = r0; i < r0 + nr; ++i) {
            const bool b = hp.bsoff[size_t(i)] >= 0;
            bnd += b;
            for (int j = 0; j < W; ++j) {
                kc.push_back(hp.ell_col[size_t(i) * W + j]);
                if (b && j < hp.bnum[size_t(i)]) bc.push_back(hp.ell_col[size_t(i) * W + j]);
            }
        }
        std::sort(kc.begin(), kc.end());
        kc.erase(std::unique(kc.begin(), kc.end()), kc.end());
        std::sort(bc.begin(), bc.end());
        bc.erase(std::unique(bc.begin(), bc.end()), bc.end());
        if (nk4 != int32_t((kc.size() + 3) / 4 * 4) || nb4 != int32_t((bc.size() + 3) / 4 * 4)) return fail(at + ": halo count");
        if (nbr != bnd) return fail(at + ": boundary rows");
        for (int32_t k = 0; k < nk4; ++k)
            if (ht.hrow[size_t(h0 + k)] != kc[std::min<size_t>(size_t(k), kc.size() - 1)]) return fail(at + ": K list");
        for (int32_t k = 0; k < nb4; ++k)
            if (ht.hrow[size_t(h0 + nk4 + k)] != bc[std::min<size_t>(size_t(k), bc.size() - 1)]) return fail(at + ": B list");
        // metadata block
        const uint32_t *M = ht.meta.data() + next_m / 4;
        const uint32_t *loc = M, *info = M + size_t(nr) * 4, *kv = M + size_t(nr) * 8, *bw = M + size_t(nr) * 24,
                       *bloc = bw + size_t(nbr) * 16;
        int32_t br = 0;
        for (int32_t g = 0; g < nr; ++g) {
            const int32_t i = r0 + g;
            const bool b = hp.bsoff[size_t(i)] >= 0;
            const std::string ar = at + " row " + std::to_string(i);
            for (int j = 0; j < W; ++j) {
                const uint32_t e = (loc[size_t(g) * 4 + j / 4] >> (8 * (j % 4))) & 0xFFu;
                const int32_t col = hp.ell_col[size_t(i) * W + j];
                if (kc[e] != col) return fail(ar + ": K index");
                if (kv[size_t(g) * 16 + j] != fbits(hp.ell_val[size_t(i) * W + j])) return fail(ar + ": K value");
            }
            const uint32_t *in = info + size_t(g) * 4;
            const int32_t nx = hp.xptr[size_t(i) + 1] - hp.xptr[size_t(i)];
            const int32_t ninj = hp.injptr[size_t(i) + 1] - hp.injptr[size_t(i)];
            if (in[0] != fbits(hp.dt / hp.mass[size_t(i)])) return fail(ar + ": dt/m");
            if ((in[1] & 0xFFu) != (b ? uint32_t(br) : 0xFFu) || int32_t((in[1] >> 8) & 0xFFu) != hp.bnum[size_t(i)] ||
                int32_t((in[1] >> 16) & 0xFFu) != nx || int32_t(in[1] >> 24) != ninj)
                return fail(ar + ": count word");
            if (int32_t(in[2]) != hp.xptr[size_t(i)]) return fail(ar + ": overflow start");
            if (int32_t(in[3]) != hp.injptr[size_t(i)]) return fail(ar + ": injection start");
            if (b) {
                for (int j = 0; j < W; ++j) {
                    if (bw[size_t(br) * 16 + j] != fbits(hp.bslot[size_t(hp.bsoff[size_t(i)]) + j])) return fail(ar + ": B value");
                    if (j < hp.bnum[size_t(i)]) {
                        const uint32_t e = (bloc[size_t(br) * 4 + j / 4] >> (8 * (j % 4))) & 0xFFu;
                        if (bc[e] != hp.ell_col[size_t(i) * W + j]) return fail(ar + ": B index");
                    }
                }
                ++br;
            }
        }
        next_row = r0 + nr;
        next_h = h0 + nk4 + nb4;
        next_m += int64_t(nr) * 96 + int64_t(nbr) * 80;
    }
    if (next_row != N) return fail("tiles do not cover the rows");
    if (size_t(next_h) != ht.hrow.size() || size_t(next_m) != ht.meta.size() * 4) return fail("trailing data");
    std::printf("OK tiles %d full %d halo rows per row %.3f\n", ht.n_tiles, full, double(ht.hrow.size()) / N);
    return 0;
}
