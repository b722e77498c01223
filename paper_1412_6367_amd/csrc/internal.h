// Internal declarations shared by the plan builder, the kernels and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/azint.h"

namespace azi {

// One unit of forward work for a workgroup.
//   rows [r0, r1) of the output, nonzeros [z0, z1) of the (device) CSR,
//   ip0 = position of row r0's start in the row-pointer array,
//   part = -1 when the tile holds whole rows and writes them directly, else
//   the partial-sum slot of this piece of a long row (one row, r1 == r0 + 1).
struct Tile {
    int32_t r0, r1, z0, z1, part, ip0, pad0, pad1;
};

// A row split over several tiles: its partial sums live in slots [p0, p1).
struct Split {
    int32_t row, p0, p1, pad;
};

// Matrix of one geometry, as built on the host.  Coefficients are kept in
// double (the builder's exact output) and rounded to the storage type on
// export or upload.
struct HostMatrix {
    int32_t npt = 0;
    int64_t npix = 0;
    double pmin = 0.0, pmax = 0.0;
    std::vector<int32_t> indptr;   // CSR, npt + 1
    std::vector<int32_t> indices;  // CSR, nnz, ascending pixel id per row
    std::vector<double> data;      // CSR, nnz
    std::vector<int32_t> colptr;   // CSC, npix + 1
    std::vector<int32_t> rowidx;   // CSC, nnz, ascending bin per pixel
    std::vector<double> cdata;     // CSC, nnz
    int64_t nnz() const { return (int64_t)indices.size(); }
};

// Geometry -> radial extents -> coefficients -> CSC and CSR.  Returns an
// AZI_* code and fills `err` on failure.
int build_matrix(const azi_geom& g, int32_t npt, int32_t unit, int32_t split,
                 const double* range2, HostMatrix& m, std::string& err);

// Appends the tile schedule of one instance.  `indptr` holds the instance's
// own row pointers (starting at 0); z_off / r_off / ip_off shift nonzeros,
// rows and row-pointer positions to the concatenated arrays.  Rows longer
// than tile_nnz are cut into nearly equal pieces with partial-sum slots
// numbered from `nparts` (updated).
void build_tiles(const int32_t* indptr, int32_t nrows, int64_t z_off, int64_t r_off,
                 int64_t ip_off, int32_t tile_nnz, std::vector<Tile>& tiles,
                 std::vector<Split>& splits, int32_t& nparts);

}  // namespace azi
