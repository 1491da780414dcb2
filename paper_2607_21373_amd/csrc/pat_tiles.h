// Work mappings of the step kernels: which tile (or sampling block) a workgroup
// takes.  Plain integer functions, compiled for the device by the kernels and for
// the host by the checks of the test suite (which define PAT_HD as `inline`).
#pragma once

#ifndef PAT_HD
#define PAT_HD __host__ __device__ inline
#endif

namespace pat {

// Workgroup b of nb is dispatched to XCD (b % 8); map it to a logical tile so that
// each XCD walks one contiguous range of rows (XCD x: floor(nb/8) tiles, one more
// for x < nb % 8).
PAT_HD int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = b & 7, k = b >> 3;
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + k;
}

// xcd_tile with each XCD's range walked from its end, for the transposed steps.
// The node order puts the rows with sensor weights at the front of each XCD's
// range, and their tiles wait on the injection chain (range, then entries, then
// data).  Dispatched last instead of first they cost the step less: on the
// 195,112-node ball 11.2 -> 10.6 us per single-RHS float64 step and 3-4% per
// float32 step of 16 or 32 RHS; the forward steps are unchanged.
PAT_HD int xcd_tile_rev(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = b & 7, k = b >> 3;
    const int len = q + (x < rem ? 1 : 0);
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + len - 1 - k;
}

// The logical tiles [0, T), T = n_rows + n_samp, of a forward step come in
// eight contiguous shares, one per XCD (share x: floor(T/8) tiles, one more
// for x < T % 8).  Each share starts with its part of the sensor-sampling
// blocks (floor(n_samp/8), one more for x < n_samp % 8), which are short and
// so are dispatched first, then its row tiles in order.  Returns the row tile,
// or n_rows + j for sampling block j.
PAT_HD int fwd_work(int l, int n_rows, int n_samp) {
    if (n_samp == 0) return l;
    const int T = n_rows + n_samp;
    const int q = T >> 3, r = T & 7;
    const int x = l < r * (q + 1) ? l / (q + 1) : r + (l - r * (q + 1)) / q;
    const int k = l - (x * q + (x < r ? x : r));
    const int sq = n_samp >> 3, sr = n_samp & 7;
    const int before = x * sq + (x < sr ? x : sr);  // sampling blocks of the shares before x
    const int mine = sq + (x < sr ? 1 : 0);
    if (k < mine) return n_rows + before + k;
    return l - before - mine;
}

// Merged launch over several meshes (Multi): workgroup b takes, on XCD b % 8, the
// next tile of the first mesh whose share on that XCD is not used up; each XCD
// takes an eighth of every mesh (as xcd_tile), walked from its end with rev (as
// xcd_tile_rev).  False for the workgroups beyond all meshes' tiles.
PAT_HD bool mesh_tile(const int *tiles, int n, int b, int *mesh, int *local, bool rev) {
    const int x = b & 7;
    int k = b >> 3;
    for (int m = 0; m < n; ++m) {
        const int q = tiles[m] >> 3, r = tiles[m] & 7;
        const int cnt = q + (x < r ? 1 : 0);
        if (k < cnt) {
            *mesh = m;
            *local = x * q + (x < r ? x : r) + (rev ? cnt - 1 - k : k);  // rev: as xcd_tile_rev
            return true;
        }
        k -= cnt;
    }
    return false;
}

// grid size of a merged launch (see Multi)
PAT_HD int multi_grid(const int *tiles, int n) {
    int c = 0;
    for (int m = 0; m < n; ++m) c += (tiles[m] >> 3) + ((tiles[m] & 7) ? 1 : 0);
    return 8 * c;
}

// HWork (the halo step kernels' work items): local index, within its XCD's range,
// of the j-th tile of workgroup k of the XCD's G8.  Unweighted, workgroup k takes
// tile k of every row of G8 tiles.  Weighted (two workgroups per CU, G8 even), every
// kRowPeriod-th row goes to the first half (k < G8 / 2), two tiles each, so that
// half takes 10 tiles for every 8 of the other.  Increasing in j.
constexpr int kRowPeriod = 9;
PAT_HD int hwork_local(int j, int G8, int k, bool weighted, bool first_half) {
    if (!weighted) return j * G8 + k;
    if (first_half) {
        const int b = j / (kRowPeriod + 1), e = j % (kRowPeriod + 1);
        return e < kRowPeriod - 1 ? (b * kRowPeriod + e) * G8 + k
                                  : (b * kRowPeriod + kRowPeriod - 1) * G8 + 2 * k + (e - (kRowPeriod - 1));
    }
    const int b = j / (kRowPeriod - 1), e = j % (kRowPeriod - 1);
    return (b * kRowPeriod + e) * G8 + k;
}

}  // namespace pat
