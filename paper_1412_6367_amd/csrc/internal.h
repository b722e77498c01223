// Internal declarations shared by the plan builder, the kernels and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

#include "../../include/azint.h"

namespace azi {

// One unit of forward work for a workgroup; rows [r0, r1) of the output,
// ip0 = position of row r0's start in the row-pointer array.
//   kTileRow:        one row (r1 == r0 + 1), nonzeros [z0, z1); part = -1
//                    writes the row, else the partial slot of this piece.
//   kTileRows:       whole rows [r0, r1), nonzeros [z0, z1), written directly.
//   kTileInterleave: piece k of z1 equal pieces of every row in [r0, r1),
//                    each row summed by its own group of lanes in lockstep
//                    with the others (neighbouring rings read the same image
//                    lines at the same time); z1 == 1 writes the rows,
//                    otherwise row r0 + i goes to slot part + i * z1 + k.
constexpr int32_t kTileRow = 0, kTileRows = 1, kTileInterleave = 2;
struct Tile {
    int32_t r0, r1, z0, z1, part, ip0, mode, k;
};

// Start of piece k of `pieces` of the row [a, b): cuts inside the row on
// multiples of 4.  Shared by the host schedule and the kernels.
__host__ __device__ inline int32_t piece_cut(int32_t a, int32_t b, int32_t k, int32_t pieces) {
    if (k <= 0) return a;
    if (k >= pieces) return b;
    const int32_t c = (int32_t)((int64_t)a + ((int64_t)(b - a) * k) / pieces) & ~3;
    return c < a ? a : c;
}

// A row split over several tiles: its partial sums live in slots [p0, p1).
struct Split {
    int32_t row, p0, p1, pad;
};

// Matrix of one geometry, as built on the host.  Coefficients are kept in
// double (the builder's exact output) and rounded to the storage type on
// export or upload.
struct HostMatrix {
    int32_t npt = 0;               // rows: npt_rad * npt_azim
    int32_t npt_rad = 0, npt_azim = 1;
    bool two_d = false;            // rows are (azimuthal wedge, radial bin) pairs
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

// Device column layout: the gather kernels read the image either in its own
// row-major pixel order, or in "ring" order -- pixels sorted by the first bin
// they feed, ties kept in pixel order -- where every bin's pixels sit in a
// few short contiguous runs.
struct RingLayout {
    int64_t used = 0;                 // pixels that feed at least one bin
    std::vector<int32_t> order;       // ring position q -> pixel id, npix
    std::vector<int32_t> pos;         // pixel id -> ring position, npix
    std::vector<int32_t> indices;     // CSR columns as ring positions, ascending per row
    std::vector<double> data;         // CSR coefficients in that order
};

void build_ring(const HostMatrix& m, RingLayout& r);

// Image tiles for moving an image into ring positions through LDS: a tile is
// a block of rows [i0, i0+th) x columns [j0, j0+tw) of one image; its pixels
// are read row-major and written to ring positions in ascending order.
//   lidx[k_off + e] = rank, among the tile's ring positions, of its e-th
//                     pixel in row-major order (e < th*tw)
//   dest[k_off + k] = the k-th smallest ring position of the tile's pixels
constexpr int32_t kStageTileH = 32, kStageTileW = 128;
struct StageTile {
    int32_t i0, j0, th, tw;  // rows / columns of the tile within its image
    int32_t w, pad;          // image width
    int64_t img_off;         // first pixel of the image in the flat array
    int64_t k_off;           // offset of the tile's entries in lidx / dest
};
static_assert(sizeof(StageTile) == 40, "stage tile layout");

// Appends the tiles of one h x w image whose ring positions are `pos`
// (offset by q_off in the flat output) starting at table offset k_off.
void build_stage_tiles(int32_t h, int32_t w, const int32_t* pos, int64_t img_off, int64_t q_off,
                       int64_t k_off, std::vector<StageTile>& tiles, std::vector<uint16_t>& lidx,
                       std::vector<int32_t>& dest);

// Geometry -> extents -> coefficients -> CSC and CSR.  npt_azim == 0 builds
// the one-dimensional matrix of npt radial bins; npt_azim >= 2 the
// two-dimensional one, row c * npt + a for wedge c of [-pi, pi) and radial
// bin a.  Returns an AZI_* code and fills `err` on failure.
int build_matrix(const azi_geom& g, int32_t npt, int32_t npt_azim, int32_t unit, int32_t split,
                 const double* range2, HostMatrix& m, std::string& err);

// Matrix blocked by image tiles: the tile layout.  Every tile of
// kStageTileH x kStageTileW pixels holds the part of the matrix its pixels
// feed, as a small CSR over the bins the tile touches, with pixel ids local
// to the tile (16 bits).  The per-(tile, bin) sums go to partial slots; bin
// b owns slots [bin_ptr[b], bin_ptr[b+1]), one per tile touching it, in tile
// order.
struct BlockTile {
    int32_t i0, j0, th, tw;  // rows / columns of the tile within its image
    int32_t w, nrows;        // image width, rows (bins) of the tile
    int64_t img_off;         // first pixel of the image in the flat array
    int64_t row_off;         // first row of the tile in the row array
    int64_t ent_off;         // first entry of the tile in the entry arrays
};
static_assert(sizeof(BlockTile) == 48, "block tile layout");
struct BlockRow {
    int32_t slot;            // partial-sum slot of this (tile, bin)
    int32_t start, end;      // entries, relative to the tile's ent_off
    int32_t bin;             // global bin
};
struct BlockMatrix {
    std::vector<BlockTile> tiles;
    std::vector<BlockRow> rows;
    std::vector<uint16_t> lp;     // local pixel id of each entry
    std::vector<double> coef;     // coefficient of each entry
    std::vector<int32_t> bin_ptr; // npt + 1 (global), partial slots per bin
};

// Appends the blocked form of one h x w image's matrix (CSC `m`) to `bm`;
// pixel offset img_off and bin offset bin_off place it in a batch.  Call
// finish_blocks once after the last instance to number the slots.
void build_blocks(const HostMatrix& m, int32_t h, int32_t w, int64_t img_off, int64_t bin_off,
                  BlockMatrix& bm);
void finish_blocks(int64_t npt_total, BlockMatrix& bm);

// Matrix grouped into bands of R consecutive bins: the band layout.  The
// entries of a band are ordered by pixel id (ties by bin), so a wavefront
// reading consecutive entries reads nearly consecutive pixels of the
// row-major image.  An entry packs its bin's offset within the band into the
// top bits of its (instance-local) pixel id.  A band's entries are cut into
// pieces; piece k of a band writes R partial sums to slots
// [slot0, slot0 + R); bin b adds its band's pieces' partials, in piece order.
constexpr int32_t kBandShift = 27;  // pixel ids below 2^27; rows in bits 27..30
struct BandPiece {
    int32_t z0, z1;          // entries
    int32_t bin0, nrows;     // first (global) bin of the band and its rows
    int32_t slot0, pad;      // partial slots slot0 .. slot0 + R - 1
    int64_t pix_off;         // first pixel of the instance
};
static_assert(sizeof(BandPiece) == 32, "band piece layout");
struct BandMatrix {
    std::vector<BandPiece> pieces;
    std::vector<int32_t> packed;  // (row in band << kBandShift) | local pixel id
    std::vector<double> coef;
    std::vector<int32_t> bin_slot;   // per global bin: first partial slot
    std::vector<int32_t> bin_count;  // per global bin: number of partials (stride R)
    int32_t nslots = 0;
};

// Appends one instance (CSC `m`) to `bm`.  Bands of R bins, pieces of at
// most piece_nnz entries (cut on multiples of 4); entries start on a
// multiple of 64 per instance.  Returns false if the image has 2^27 pixels
// or more.
bool build_bands(const HostMatrix& m, int32_t R, int32_t piece_nnz, int64_t pix_off,
                 int64_t bin_off, BandMatrix& bm);
// The pieces, slots and per-bin slot ranges of one instance whose band b
// holds entries [base + start[b], base + start[b + 1]) (the second half of
// build_bands, also used when the entries were ordered on the device).
void band_pieces(const int64_t* start, int32_t nbands, int32_t npt, int32_t R, int32_t piece_nnz,
                 int64_t base, int64_t pix_off, int64_t bin_off, BandMatrix& bm);

// Run encoding of the band layout (bands of kRunRows bins).  A run is the
// stretch of one pixel's entries inside one band (consecutive bins): one
// word pix | first row << kBandShift | (count - 1) << kRunCountShift.  Runs
// of a band are in pixel order; every band, and so every piece, starts on a
// multiple of 64 runs (the padding words are -1).  The coefficients of the 64 runs of group g start at
// gbase[g], slot-major: the first coefficient of each run in run order,
// then the second of the runs that have one, and so on.  A wavefront takes
// one group and finds every lane's coefficients from the counts alone.
// Pieces (z0, z1 in runs) and slots are as in the band layout.
constexpr int32_t kRunRows = 4;
constexpr int32_t kRunCountShift = 29;
struct RunMatrix {
    std::vector<BandPiece> pieces;
    std::vector<int32_t> runs;
    std::vector<int32_t> gbase;
    std::vector<double> coef;
    std::vector<int32_t> bin_slot, bin_count;
    int32_t nslots = 0;
};
// Appends the run encoding of one instance (CSC `m`; its pixels start at
// pix_off, its bins at bin_off of the batch) to `rm`, with pieces of at most
// piece_runs runs (rounded down to a multiple of 64).  Returns false if the
// image has 2^27 pixels or more, the runs or coefficients would not fit
// int32 positions, or waves exceeds 32.
// With `scale` (npix values), every coefficient of pixel p is multiplied by
// scale[p] (rounded once) as it is stored.
// waves > 1: the pieces are instead cut for workgroups of `waves`
// neighbouring bands over common stretches of image rows: entry
// t * waves + w of rm.pieces is band w of workgroup t (z0 == z1 and slot0 ==
// -1 past the last band).  Each band's runs are cut on multiples of 64: a
// group of 64 runs belongs to the stretch that holds its first pixel.  The
// stretches are cut in pixel order so that no band has more than a bound of
// groups of 64 runs in one (the greedy cut, which gives the fewest
// stretches), then made as even as their number allows (the smallest bound
// giving no more).  The bound is piece_runs / 64 groups or, with
// round_tiles > 0 (the workgroups a device keeps resident at once), the
// smallest that keeps the instance's workgroups within k * round_tiles, for
// the fewest rounds k that bring the bound to kRoundRuns runs or less: each
// round's workgroups then take as nearly the same work as the bands allow.
constexpr int64_t kRoundRuns = 2048;
bool build_runs(const HostMatrix& m, int32_t piece_runs, int64_t pix_off, int64_t bin_off,
                RunMatrix& rm, const double* scale = nullptr, int32_t waves = 1,
                int64_t round_tiles = 0);

// Matrix-free ("fused") schedule: the image cut into kFusedH x kFusedW
// tiles; tile t feeds the bin window [wlo, wlo + nwin) and writes the partial
// sums of bin wlo + k to slot slots[slot_off + k]; bin b owns slots
// [bin_ptr[b], bin_ptr[b + 1]), one per tile whose window holds it, in tile
// order.  Windows come from the pixel-major entries of the plan's matrix.
constexpr int32_t kFusedH = 8, kFusedW = 64;
struct FusedTile {
    int32_t i0, j0, th, tw;
    int32_t wlo, nwin;
    int64_t slot_off;
};
static_assert(sizeof(FusedTile) == 32, "fused tile layout");
void build_fused(const HostMatrix& m, int32_t h, int32_t w, std::vector<FusedTile>& tiles,
                 std::vector<int32_t>& slots, std::vector<int32_t>& bin_ptr);

// Appends the tile schedule of one instance.  `indptr` holds the instance's
// own row pointers (starting at 0); z_off / r_off / ip_off shift nonzeros,
// rows and row-pointer positions to the concatenated arrays.  Rows longer
// than tile_nnz are cut into nearly equal pieces with partial-sum slots
// numbered from `nparts` (updated).
// `band` > 1 groups runs of `band` consecutive rows longer than
// tile_nnz / band into kTileInterleave tiles of about tile_nnz nonzeros.
void build_tiles(const int32_t* indptr, int32_t nrows, int64_t z_off, int64_t r_off,
                 int64_t ip_off, int32_t tile_nnz, int32_t band, std::vector<Tile>& tiles,
                 std::vector<Split>& splits, int32_t& nparts);

}  // namespace azi
