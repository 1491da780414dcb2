// Internal declarations shared by the host setup (pat_setup.cpp) and the
// device code (pat_api.hip, pat_kernels.hip) of libpat.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pat.h"

namespace pat {

// Host-side assembled problem, all node indices in the library's internal order.
struct HostProblem {
    int32_t n = 0;          // nodes
    int32_t n_obs = 0;
    int32_t n_steps = 0;
    int64_t n_tets = 0;
    double dt = 0.0;
    // stiffness pattern (CSR, columns ascending) shared by K and K1
    std::vector<int32_t> rowptr, col;
    std::vector<double> kval, k1val;
    // boundary mass: for a boundary row i, boff[i] >= 0 and B(i, col[k]) = bval[boff[i] + k - rowptr[i]]
    // for k in [rowptr[i], rowptr[i+1]); interior rows have boff[i] = -1
    std::vector<int32_t> boff;
    std::vector<double> bval;
    int64_t nnz_b = 0;
    int32_t n_boundary = 0;
    int32_t max_row = 0;
    std::vector<double> mass;          // lumped mass diag(M 1)
    // sensors: 4 (node, weight) pairs each; node-coincident sensors use one weight 1
    std::vector<int32_t> snode;        // [n_obs][4]
    std::vector<double> sw;            // [n_obs][4]
    // transpose of the sensor operator as a node-major CSR: node i receives
    // sum_e injw[e] * yhat[injs[e]] for e in [injptr[i], injptr[i+1])
    std::vector<int32_t> injptr, injs;
    std::vector<double> injw;
    // Padded row layout of K used by the time-step kernels: entry j < kEll of row i
    // at i*kEll + j (padding: column i, value 0); entries beyond kEll of a long row
    // in a small CSR (xptr, xcol, xval).  Boundary rows keep their B values per
    // slot: B(i, slot) = bslot[bsoff[i] + slot], slot < kEll + (xptr[i+1]-xptr[i]).
    static constexpr int kEll = 16;
    std::vector<int32_t> ell_col, xptr, xcol, bsoff;
    std::vector<double> ell_val, xval, bslot;
    // Boundary rows list their slots with a nonzero B first: B(i, slot) = 0 for
    // slot >= bnum[i] (bnum = 0 for interior rows).
    std::vector<int32_t> bnum;
    // internal <-> user numbering: perm[internal] = user, iperm[user] = internal
    std::vector<int32_t> perm, iperm;
    double lambda_max = 0.0;
};

// Assemble and validate; returns PAT_OK or an error with a message in *err.
pat_status build_host_problem(const pat_problem_desc &d, HostProblem &hp, std::string &err);

// Build the padded row layout (ell_*, x*, bs*) from the CSR arrays.
void build_padded_rows(HostProblem &hp);

// Halo tiles of the float32 step kernels whose RHS block rows are 256-byte
// multiples.  Consecutive rows (a compact cluster of the node order) are cut
// greedily into tiles of at most kRows rows whose halo, the distinct rows that
// the tile's padded slots refer to (K rows) plus the distinct rows its boundary
// slots refer to (B rows), each padded to a multiple of 4, holds at most kMax
// rows.  Per tile: a descriptor, the halo's row list and one metadata block
// that the kernels copy into LDS with the halo (96 B per row, 80 more per
// boundary row):
//   loc[nr][16]   uint8:  K-local index of each slot (kMax < 256)
//   info[nr][4]   uint32: dt/m (float bits); boundary row (0xFF: none) | bnum << 8 |
//                         (xptr[i+1] - xptr[i]) << 16 | (injptr[i+1] - injptr[i]) << 24;
//                         xptr[i]; injptr[i]
//   kv[nr][16]    float:  the slot values of K
//   bw[nbr][16]   float:  the slot values of B of the tile's boundary rows
//   bloc[nbr][16] uint8:  B-local index of each of their first min(bnum, 16) slots
// A mesh with a count beyond its byte (bnum, overflow entries or injections of a
// row above 255) gets no halo tiles and runs on the vector-lane kernels.
struct HaloTiles {
    static constexpr int kRows = 32;
    static constexpr int kMax = 132;
    static constexpr int kMetaBytes = kRows * (16 + 16 + 64 + 64 + 16);
    static constexpr int kNrBits = 7;  // descriptor field of the rows and of the boundary rows
    static_assert(kRows < (1 << kNrBits) && kMax < 256 && kMax % 4 == 0, "descriptor fields");
    int32_t n_tiles = 0;
    // [n_tiles][4]: first row, first halo entry, metadata offset (16-byte units),
    // rows | K rows << kNrBits | B rows << (kNrBits + 8) | boundary rows << (kNrBits + 16)
    // (metadata bytes: 96 per row + 80 per boundary row)
    std::vector<int32_t> desc;
    std::vector<int32_t> hrow;
    std::vector<uint32_t> meta;
};
void build_halo_tiles(const HostProblem &hp, HaloTiles &ht);


// Largest eigenvalue of M_L^{-1} K by power iteration on M^{-1/2} K M^{-1/2}.
double estimate_lambda_max(const HostProblem &hp, int iters);

// Growth test of the explicit step (with the boundary term) in float64 on the host:
// returns the ratio E_final / E_initial of the discrete energy after `steps` steps.
double energy_growth(const HostProblem &hp, int steps);

}  // namespace pat
