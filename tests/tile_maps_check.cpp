// Host check of the step kernels' work mappings (pat_tiles.h): every launch
// shape maps its workgroups one to one onto the tiles (and sampling blocks) it
// must cover, with the per-XCD ranges and orders the kernels rely on.  Prints
// "OK ..." and exits 0, or prints the first failure and exits 1.
#define PAT_HD inline
#include "pat_tiles.h"

#include <cstdio>
#include <string>
#include <vector>

namespace {
int fail(const std::string &what) {
    std::printf("FAIL %s\n", what.c_str());
    return 1;
}
}  // namespace

int main() {
    using namespace pat;
    long checks = 0;
    // xcd_tile / xcd_tile_rev: bijections on [0, nb); XCD x's workgroups (b % 8 == x)
    // cover one contiguous range, in increasing (xcd_tile) or decreasing (rev) order
    for (int nb = 1; nb <= 3000; ++nb) {
        for (int rev = 0; rev < 2; ++rev) {
            std::vector<int> hit(size_t(nb), 0);
            for (int x = 0; x < 8; ++x) {
                int prev = -1, lo = 1 << 30, hi = -1, cnt = 0;
                for (int b = x; b < nb; b += 8) {
                    const int t = rev ? xcd_tile_rev(b, nb) : xcd_tile(b, nb);
                    if (t < 0 || t >= nb) return fail("xcd tile out of range, nb " + std::to_string(nb));
                    ++hit[size_t(t)];
                    if (prev >= 0 && (rev ? t != prev - 1 : t != prev + 1))
                        return fail("xcd range order, nb " + std::to_string(nb));
                    prev = t;
                    lo = t < lo ? t : lo;
                    hi = t > hi ? t : hi;
                    ++cnt;
                }
                if (cnt > 0 && hi - lo + 1 != cnt) return fail("xcd range not contiguous, nb " + std::to_string(nb));
            }
            for (int t = 0; t < nb; ++t)
                if (hit[size_t(t)] != 1) return fail("xcd tile hit count, nb " + std::to_string(nb));
            ++checks;
        }
    }
    // fwd_work: a bijection from [0, n_rows + n_samp) onto the row tiles and the
    // sampling blocks, each XCD's share starting with its sampling blocks
    for (int n_rows = 1; n_rows <= 700; n_rows += 3)
        for (int n_samp = 0; n_samp <= 40; ++n_samp) {
            const int T = n_rows + n_samp;
            std::vector<int> hit(size_t(T), 0);
            for (int l = 0; l < T; ++l) {
                const int w = fwd_work(l, n_rows, n_samp);
                if (w < 0 || w >= T) return fail("fwd_work out of range");
                ++hit[size_t(w)];
            }
            for (int w = 0; w < T; ++w)
                if (hit[size_t(w)] != 1) return fail("fwd_work hit count, rows " + std::to_string(n_rows));
            const int q = T >> 3, r = T & 7;
            for (int x = 0, l0 = 0; x < 8; ++x) {  // within a share: sampling blocks, then rows
                const int len = q + (x < r ? 1 : 0);
                bool rows_seen = false;
                for (int l = l0; l < l0 + len; ++l) {
                    const bool samp = fwd_work(l, n_rows, n_samp) >= n_rows;
                    if (samp && rows_seen) return fail("fwd_work: a sampling block after a row tile");
                    rows_seen = rows_seen || !samp;
                }
                l0 += len;
            }
            ++checks;
        }
    // mesh_tile: over multi_grid(tiles) workgroups, every (mesh, tile) exactly once
    for (int n = 1; n <= 4; ++n)
        for (int seed = 0; seed < 400; ++seed) {
            int tiles[4];
            unsigned v = 2654435761u * unsigned(seed + 1) + unsigned(n);
            for (int m = 0; m < n; ++m) {
                v = v * 1103515245u + 12345u;
                tiles[m] = 1 + int((v >> 8) % 300u);
            }
            const int grid = multi_grid(tiles, n);
            for (int rev = 0; rev < 2; ++rev) {
                std::vector<std::vector<int>> hit(static_cast<size_t>(n));
                for (int m = 0; m < n; ++m) hit[size_t(m)].assign(size_t(tiles[m]), 0);
                for (int b = 0; b < grid; ++b) {
                    int m = -1, local = -1;
                    if (!mesh_tile(tiles, n, b, &m, &local, rev != 0)) continue;
                    if (m < 0 || m >= n || local < 0 || local >= tiles[m]) return fail("mesh_tile out of range");
                    ++hit[size_t(m)][size_t(local)];
                }
                for (int m = 0; m < n; ++m)
                    for (int t = 0; t < tiles[m]; ++t)
                        if (hit[size_t(m)][size_t(t)] != 1) return fail("mesh_tile hit count");
                ++checks;
            }
        }
    // hwork_local: the tiles [0, ntx) of one XCD's range split over its G8 workgroups,
    // each tile to exactly one, with the per-workgroup count the kernel derives
    // (per_c: the first j with local(j) >= ntx; local increasing in j)
    for (int G8 = 1; G8 <= 64; ++G8)
        for (int weighted = 0; weighted < 2; ++weighted) {
            if (weighted && G8 % 2) continue;  // the kernels weight only even G8
            for (int ntx = 0; ntx <= 40 * G8 + 13; ntx += (G8 < 8 ? 1 : 7)) {
                std::vector<int> hit(size_t(ntx), 0);
                for (int k = 0; k < G8; ++k) {
                    const bool first_half = 2 * k < G8;
                    int per_c = 0, prev = -1;
                    while (true) {
                        const int t = hwork_local(per_c, G8, k, weighted != 0, first_half);
                        if (t <= prev) return fail("hwork_local not increasing, G8 " + std::to_string(G8));
                        if (t >= ntx) break;
                        ++hit[size_t(t)];
                        prev = t;
                        ++per_c;
                    }
                }
                for (int t = 0; t < ntx; ++t)
                    if (hit[size_t(t)] != 1)
                        return fail("hwork tile hit count, G8 " + std::to_string(G8) + " ntx " + std::to_string(ntx));
                ++checks;
            }
        }
    std::printf("OK %ld launch shapes\n", checks);
    return 0;
}
