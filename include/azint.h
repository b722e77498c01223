/*
 * azint.h -- C ABI of the MI355X (gfx950) azimuthal-integration library.
 *
 * The library reduces a 2-D detector image to a 1-D profile over the radial
 * coordinate, or to a 2-D (azimuth x radius) map, with pixel splitting
 * (Kieffer & Ashiotis, "PyFAI: a Python library for high performance
 * azimuthal integration on GPU", EuroSciPy 2014).  The image is corrected
 * pixel by pixel (Section 6.4), then each output bin b receives
 *
 *     W_b = sum_p A_bp x_p      (weighted histogram)
 *     U_b = sum_p A_bp          (unweighted histogram)
 *     I_b = W_b / U_b           (their ratio, the profile)
 *
 * where A is the pixel-to-bin coefficient matrix of Section 4, built once
 * per geometry and applied per frame as a CSR sparse-matrix / dense-vector
 * product in "gather" form (Section 5.2, 5.2.1).  Every per-frame call
 * below works on one- and two-dimensional plans alike: a plan's bins are
 * its "npt" rows (npt_rad * npt_azim for a two-dimensional plan).
 *
 * Conventions shared by every call:
 *   - Return value: AZI_OK (0) on success, a negative AZI_E* code otherwise;
 *     azi_last_error() then returns a message for the calling thread.  A
 *     failed call leaves its outputs unspecified and its objects unchanged.
 *   - "device" pointers are HIP device addresses on the plan's device;
 *     "host" pointers are ordinary CPU memory.  The caller owns every data
 *     buffer it passes; the library owns plans, batches and graphs (their
 *     device matrices, tile schedules and work buffers) and frees them in
 *     the matching *_destroy call.
 *   - Images are row-major h x w (pixel id p = i*w + j).  Arrays of a plan's
 *     storage type hold float (AZI_F32) or double (AZI_F64) values.
 *   - Per-frame calls (azi_correct, azi_integrate1d*, azi_batch_forward,
 *     azi_batch_backward, azi_graph_launch) enqueue work on the given HIP
 *     stream (NULL = the null stream) and return without synchronising; they
 *     allocate nothing, so they may be captured into a HIP graph.  They use
 *     work buffers owned by the plan or batch: two calls on one plan or batch
 *     that overlap in time (different streams) race on those buffers.
 *   - Integer and index work is exact; floating-point sums are deterministic
 *     run to run for a fixed tiling (no floating-point atomics).
 */
#ifndef AZINT_H
#define AZINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AZI_ABI_VERSION 1

/* Error codes. */
#define AZI_OK          0
#define AZI_EINVAL     -1  /* bad argument: null pointer, size, enum, range  */
#define AZI_ENOMEM     -2  /* host or device allocation failed              */
#define AZI_EOVERFLOW  -3  /* a count does not fit int32 (nnz, pixels, bins) */
#define AZI_EDEVICE    -4  /* HIP runtime error or no usable device          */
#define AZI_ESTATE     -5  /* object not in the state the call needs         */

/* Output coordinate (Section 3, coordinate list). */
#define AZI_UNIT_R_M     0  /* radius in metres                     */
#define AZI_UNIT_R_MM    1  /* radius in millimetres                */
#define AZI_UNIT_2TH_RAD 2  /* scattering angle 2theta = atan(r/d)  */
#define AZI_UNIT_2TH_DEG 3  /* the same in degrees                  */
#define AZI_UNIT_Q_NM    4  /* q = 4 pi sin(2theta/2) / lambda, 1/nm */

/* Pixel splitting: AZI_SPLIT_NONE, whole pixels by their midpoint (Section
 * 3.3 histogram); AZI_SPLIT_BBOX, the radial bounding box of each pixel
 * (Section 4.1); AZI_SPLIT_FULL, the area of the pixel's corner
 * quadrilateral in (output unit, azimuth) space with straight edges, shared
 * by area (Section 4.2) -- pixels holding the beam centre use the bounding
 * box, where that quadrilateral is undefined. */
#define AZI_SPLIT_NONE 0
#define AZI_SPLIT_BBOX 1
#define AZI_SPLIT_FULL 2

/* Element types. */
#define AZI_I16 0
#define AZI_U16 1
#define AZI_I32 2
#define AZI_U32 3
#define AZI_F32 4
#define AZI_F64 5

/* Accumulation of the per-bin sums (Section 5.2.2). */
#define AZI_ACC_F64     0  /* double accumulators (any storage type)            */
#define AZI_ACC_KAHAN32 1  /* float with Kahan compensation (AZI_F32 storage only) */

/*
 * Detector geometry: a planar detector orthogonal to the beam (Section 3).
 * Pixel (i, j) covers [j, j+1] x [i, i+1] in pixel units; the beam centre
 * is given in those units (column center_x_px, row center_y_px).  Pixel
 * sizes, distance and wavelength are in metres.
 */
typedef struct azi_geom {
    int32_t h, w;
    double pixel_y_m, pixel_x_m;
    double center_y_px, center_x_px;
    double dist_m;
    double wavelength_m;
} azi_geom;

typedef struct azi_plan azi_plan;
typedef struct azi_batch azi_batch;
typedef struct azi_graph azi_graph;

/* Library ABI version (AZI_ABI_VERSION of the build). */
int32_t azi_version(void);

/* Message of the last failed call on this thread ("" if none).  The string
 * stays valid until the next call on this thread. */
const char* azi_last_error(void);

/*
 * Build the coefficient matrix of one geometry on the host (Section 4.1 for
 * AZI_SPLIT_BBOX, 4.2 for AZI_SPLIT_FULL, 3.3 for AZI_SPLIT_NONE; Section
 * 5.2 turns the per-pixel contributions into a per-bin gather).  For every pixel the
 * radial extent [lo, hi] of the pixel square is mapped to the output unit;
 * bins are npt uniform intervals over range2 = {min, max} (host, may be NULL
 * for the data's own range: [min lo, max hi] with splitting, the range of
 * pixel-centre values without); a box partly outside the range keeps only
 * its inside share, normalised by its full width; the last bin is closed.
 * dtype (AZI_F32 / AZI_F64) is the storage type of coefficients, images and
 * outputs; accum one of AZI_ACC_*.  Nothing is placed on a device yet (see
 * azi_plan_upload).  Errors: AZI_EINVAL (null geom/out, h or w < 1, npt < 1,
 * non-positive pixel size/distance/wavelength, min >= max, bad enum,
 * Kahan accumulation with AZI_F64), AZI_EOVERFLOW (pixels or nnz >= 2^31).
 */
int azi_plan_create(const azi_geom* geom, int32_t npt, int32_t unit, int32_t split,
                    const double* range2, int32_t dtype, int32_t accum, azi_plan** out);

/*
 * Two-dimensional integration (Section 4, where pixel splitting is said to
 * matter most for the 2-D case): bins are npt_azim equal wedges of the azimuth chi =
 * atan2(y, x) over the periodic circle [-pi, pi) (x along pixel columns, y
 * along pixel rows, from the beam) times npt_rad radial bins chosen as in
 * azi_plan_create; bin (wedge c, radial bin a) is row c * npt_rad + a, so
 * every output is an npt_azim x npt_rad row-major map.  AZI_SPLIT_NONE puts a
 * pixel whole into the bin of its midpoint; AZI_SPLIT_BBOX gives bin (a, c)
 * the product of the radial share of azi_plan_create and the azimuthal
 * share of the box [chi_lo, chi_hi] spanned by the pixel's corner azimuths
 * (the whole circle, evenly, for a pixel holding the beam); AZI_SPLIT_FULL
 * the area of the corner quadrilateral inside the bin's rectangle over the
 * quadrilateral's area (bounding box for a pixel holding the beam).
 * Errors as azi_plan_create, plus AZI_EINVAL for npt_azim < 2 and
 * AZI_EOVERFLOW if npt_rad * npt_azim >= 2^31.
 */
int azi_plan_create2d(const azi_geom* geom, int32_t npt_rad, int32_t npt_azim, int32_t unit,
                      int32_t split, const double* range2, int32_t dtype, int32_t accum,
                      azi_plan** out);

/*
 * Build a one-dimensional plan on a device (Section 5.2 scatter-to-gather,
 * Section 5.2.1 CSR, done by the GPU): per-pixel extents and entries are
 * computed by device kernels from the same operations as azi_plan_create,
 * the pixel-major (CSC) order comes from a scan of the per-pixel counts and
 * the bin-major (CSR) and band orders from a stable radix sort by bin, so
 * the matrix is the one azi_plan_create builds (bit for bit with
 * AZI_UNIT_R_M / _R_MM and the bounding box or no split; coefficients to
 * rounding otherwise).  The plan comes back uploaded to `device` in the band
 * layout, ready for per-frame calls, with a host copy of its matrix for the
 * export and layout calls.  Work is enqueued on `stream` (NULL = null stream)
 * and the call synchronises it before returning.  Errors as azi_plan_create,
 * plus AZI_EDEVICE (no such device, HIP failure) and AZI_ENOMEM (device
 * memory: about 50 bytes per nonzero during the build).
 */
int azi_plan_create_device(const azi_geom* geom, int32_t npt, int32_t unit, int32_t split,
                           const double* range2, int32_t dtype, int32_t accum, int32_t device,
                           void* stream, azi_plan** out);

/*
 * The two-dimensional plan of azi_plan_create2d (Section 4, radius x
 * azimuth) built on a device by the same kernels as azi_plan_create_device:
 * per-pixel entries from the operations of the host builder (the radial
 * shares bit for bit with AZI_UNIT_R_M / _R_MM; the azimuths from the
 * device's atan2, which may differ from the C library's by an ulp, so a
 * coefficient at a wedge edge can differ by rounding and a sliver entry of
 * a few ulps can appear or vanish), the row-major (CSR) order from the
 * stable radix sort by row.  The plan comes back uploaded to `device` in
 * the pixel layout with the two-dimensional default tiling, with a host
 * copy of its matrix.  Errors as azi_plan_create2d and
 * azi_plan_create_device.
 */
int azi_plan_create2d_device(const azi_geom* geom, int32_t npt_rad, int32_t npt_azim,
                             int32_t unit, int32_t split, const double* range2, int32_t dtype,
                             int32_t accum, int32_t device, void* stream, azi_plan** out);

/* Free a plan and its device memory.  NULL is accepted (no-op). */
int azi_plan_destroy(azi_plan* plan);

/* Sizes of a plan (host outputs, each may be NULL): npt = bins (rows of
 * the matrix, npt_rad * npt_azim for a two-dimensional plan).  range2
 * receives the radial {min, max} actually used. */
int azi_plan_info(const azi_plan* plan, int32_t* npt, int64_t* npix, int64_t* nnz,
                  double* range2);

/* Radial bins npt_rad and azimuthal wedges npt_azim (0 for a
 * one-dimensional plan); host outputs, each may be NULL. */
int azi_plan_shape(const azi_plan* plan, int32_t* npt_rad, int32_t* npt_azim);

/* Radial bin centres min + (a + 0.5) * (max - min) / npt_rad, npt_rad
 * doubles (host). */
int azi_plan_positions(const azi_plan* plan, double* positions);

/* Wedge centres -pi + (c + 0.5) * 2 pi / npt_azim in radians, npt_azim
 * doubles (host).  AZI_ESTATE for a one-dimensional plan. */
int azi_plan_azimuths(const azi_plan* plan, double* chi);

/* Copy the matrix out in CSR form (host buffers): data[nnz] of the storage
 * type, indices[nnz] pixel ids ascending within a row, indptr[npt + 1]; the
 * triple is accepted as-is by scipy.sparse.csr_matrix (Section 5.2.1). */
int azi_plan_export_csr(const azi_plan* plan, void* data, int32_t* indices,
                        int32_t* indptr);

/* Copy the matrix out in pixel-major (CSC) form (host buffers): data[nnz],
 * bins[nnz] ascending within a pixel, colptr[npix + 1]. */
int azi_plan_export_csc(const azi_plan* plan, void* data, int32_t* bins, int32_t* colptr);

/*
 * Launch and tile schedule of the forward kernel (tuning only: results
 * change at most in the order of the floating-point additions, and, for
 * the stage, by the one rounding of the fused or folded correction).  A
 * new plan starts at tile_nnz 0, block 256, variant 5, grid 0, band 16,
 * stage AZI_STAGE_FOLD_SUM (plans built on the device, which start in the band
 * layout: band 4; two-dimensional plans: 4096, 256, 1, 0, 1,
 * AZI_STAGE_GATHER); a new batch at the same tiling.
 *   tile_nnz  most nonzeros one workgroup sums per tile (64..16384, a
 *             multiple of 64); rows longer than that are cut into pieces
 *             whose sums are added in order by a small fix-up kernel.
 *             0: sized by the library.  Run layout with band 16 or 32
 *             (one-dimensional or 2-D plans): each group of bands' common
 *             stretches are cut so that no band has more than a bound of
 *             runs in one, the stretches of a group as even as their number
 *             allows, with the smallest bound that keeps the workgroups
 *             within k rounds of what the device holds at once (CUs x 8 for
 *             band 16, x 4 for band 32), k the fewest rounds whose bound is
 *             2048 runs or less: every resident workgroup takes about the
 *             same work.  Other layouts, and every layout of a batch: 2048
 *             below 2^22 nonzeros (of the instance, in a batch), else 4096.
 *   block     threads per workgroup: 64, 128, 256 or 512.
 *   variant   load scheme, 0..AZI_NUM_VARIANTS-1: 0 four consecutive
 *             nonzeros per lane, 2 loads in flight; 4 the same with 4 in
 *             flight; 1, 2, 6 lane-strided (one gather instruction reads
 *             consecutive nonzeros of a row) with 4, 8, 16 in flight,
 *             2 loading the coefficients non-temporally; 3 and 5 as 2
 *             and 6 with non-temporal loads of the whole matrix.
 *   grid      0: one workgroup per tile; > 0: that many persistent
 *             workgroups walk the tiles.
 *   band      > 1: pieces of up to `band` consecutive long rows are
 *             interleaved, so tiles that run together read the same part of
 *             neighbouring rings; 0 or 1: rows one after the other.  Band
 *             layout: bins per band (4, 8 or 16).  Run layout: 16 or 32
 *             puts 4 or 8 neighbouring bands of 4 bins in one workgroup (one
 *             wavefront per band, over common stretches of image rows, so
 *             that they share the gathered image lines in the CU's cache;
 *             the workgroup then has 256 or 512 threads whatever `block`
 *             says); other values, one band per workgroup of `block`.
 *   stage     how an image is brought into ring positions (ring layout only):
 *             AZI_STAGE_GATHER reads each ring position's pixel; _SCATTER
 *             reads row-major and writes each pixel's ring position;
 *             _TILE reads 32x128-pixel tiles row-major and writes them out in
 *             ring order through LDS.  AZI_STAGE_FUSE (band and run layouts): the
 *             raw-frame calls (azi_integrate1d_raw, azi_batch_forward_raw)
 *             run one band kernel that casts and corrects every pixel it
 *             gathers as (raw - dark) * (1 / norm), dark and the reciprocal
 *             of norm (formed once per correction set, held as one pair per
 *             pixel: 2 storage values) read in one load, and never write the
 *             corrected image (256 threads per workgroup).  The product by
 *             the rounded reciprocal differs from the quotient of
 *             azi_correct by at most one rounding per pixel.  azi_plan_stage
 *             and the staged call keep the two passes.
 *             AZI_STAGE_FOLD (run layout; the band layout takes it as
 *             AZI_STAGE_FUSE): as AZI_STAGE_FUSE, but 1 / norm is folded
 *             into the coefficients when the corrections are set (a second
 *             copy of the coefficients, each multiplied by its pixel's
 *             1 / norm and rounded once) and each run of the run encoding
 *             keeps its pixel's dark value beside its word (in 16 bits when
 *             every dark value is an integer in [0, 65535], as a float when
 *             every one is a float, else in the storage type: exact
 *             conversions, the same bits), so the raw count is the only
 *             gathered value: the kernel forms
 *             A_bp * (raw - dark) with A_bp carrying 1 / norm, the same sum
 *             in another order, one rounding per product away from the
 *             quotient of azi_correct.  U, which does not depend on the
 *             image, is summed once from the unfolded coefficients at that
 *             point and written with every frame.
 *             AZI_STAGE_FOLD_SUM (run layout; the band layout takes it as
 *             AZI_STAGE_FUSE): as AZI_STAGE_FOLD, but, for plans that
 *             accumulate in float64, the dark term of W does not depend on
 *             the frame either: D_b = sum_p A_bp * dark_p (A_bp carrying
 *             1 / norm) is summed once per correction set, in the
 *             per-frame order, and the frame's W is sum_p A_bp * raw_p - D_b,
 *             so no dark value is read per frame.  The subtraction moves the
 *             rounding error's scale from sum_p A_bp |raw_p - dark_p| to
 *             sum_p A_bp (|raw_p| + |dark_p|): the error grows with the ratio
 *             of dark current to signal in a bin, about linearly: in
 *             float64, 3.1e-14 of sum_p A_bp |x_p| measured at a ratio of
 *             100 and 3.2e-13 at 1000, so the 1e-12 tolerance is reached
 *             near 3000.
 *             Plans
 *             with Kahan float sums keep the dark value per run (as
 *             AZI_STAGE_FOLD).
 */
#define AZI_NUM_VARIANTS 7
#define AZI_STAGE_GATHER 0
#define AZI_STAGE_SCATTER 1
#define AZI_STAGE_TILE 2
#define AZI_STAGE_FUSE 3
#define AZI_STAGE_FOLD 4
#define AZI_STAGE_FOLD_SUM 5
typedef struct azi_tiling {
    int32_t tile_nnz, block, variant, grid, band, stage;
} azi_tiling;

/* Set a plan's tiling (host struct).  Takes effect at the next
 * azi_plan_upload, or immediately if already uploaded (the call then
 * synchronises the device).  AZI_EINVAL for values outside the ranges above. */
int azi_plan_set_tiling(azi_plan* plan, const azi_tiling* tiling);

/* A plan's tiling and, if on a device, its number of tiles (may be NULL). */
int azi_plan_get_tiling(const azi_plan* plan, azi_tiling* tiling, int32_t* ntiles);

/* Host-side view of the tile schedule a tiling gives (no device needed;
 * for inspection and tests).  Each tile is 8 int32: {row_begin, row_end,
 * nnz_begin, nnz_end, partial_slot (-1 = whole rows), rowptr_pos, 0, 0};
 * each split row 4 int32: {row, slot_begin, slot_end, 0}.  Pass NULL arrays
 * to query the counts first. */
int azi_plan_tile_schedule(const azi_plan* plan, const azi_tiling* tiling, int32_t* ntiles,
                           int32_t* tiles, int32_t* nsplits, int32_t* splits);

/* Host-side view of the run encoding (AZI_LAYOUT_RUN) of a one-dimensional
 * or 2-D plan's matrix with pieces of tile_nnz / 2 runs (tile_nnz 0: sized
 * as the tiling's tile_nnz 0 sizes them on the plan's device, or on 256 CUs
 * for a plan without one; no device needed;
 * for inspection and tests).  Host buffers, any of them NULL to skip:
 *   runs[nruns]      pixel | first row in the band << 27 | (count - 1) << 29
 *                    per run, -1 for the padding that starts every band on a
 *                    multiple of 64 runs;
 *   gbase[nruns/64]  first coefficient of each group of 64 runs;
 *   coef[nnz]        the coefficients (double), slot-major per group: the
 *                    first coefficient of each run in run order, then the
 *                    second of the runs that have one, and so on;
 *   pieces[8 * npieces] int32 {run_begin, run_end, first bin of the band,
 *                    rows of the band, first partial slot, 0, 0, 0}; with
 *                    the plan's tiling band 16 or 32, the workgroups' entries
 *                    (4 or 8 per workgroup, one per band, slot -1 past the
 *                    last band);
 *   bin_slot[npt], bin_count[npt]  each bin's first partial slot and count
 *                    (slots first, first + 4, ...).
 * nruns / npieces (may be NULL) receive the counts.  AZI_EOVERFLOW for
 * images of 2^27 pixels or more, AZI_EINVAL for a tile_nnz other than 0
 * outside [64, 16384]. */
int azi_plan_run_schedule(const azi_plan* plan, int32_t tile_nnz, int64_t* nruns, int32_t* runs,
                          int32_t* gbase, double* coef, int32_t* npieces, int32_t* pieces,
                          int32_t* bin_slot, int32_t* bin_count);

/*
 * Device layout of the matrix (default AZI_LAYOUT_RUN, or AZI_LAYOUT_PIXEL
 * for images of 2^27 pixels or more; plans built on the device start in
 * AZI_LAYOUT_BAND; two-dimensional plans default to AZI_LAYOUT_PIXEL with
 * tile_nnz 4096, variant 2, band 1, their rows being short).  AZI_LAYOUT_PIXEL: the gather kernels
 * read the image in its row-major pixel order.  AZI_LAYOUT_RING:
 * the matrix columns are renumbered so that pixels are sorted by the first
 * bin they feed (ties in pixel order); every bin then reads its pixels from
 * a few short contiguous runs.  The renumbering is applied to the image by
 * the per-frame correction pass (or a plain permutation pass for an image
 * that is already corrected), so callers always pass row-major images and
 * the results are the same sums (Section 5.2 gather) in another order.
 * AZI_LAYOUT_TILE: the matrix is blocked by image tiles of 32 x 128 pixels.
 * One workgroup per tile reads the tile's pixels once, coalesced, applying
 * the cast and correction on the way, keeps them in LDS, and gathers every
 * bin the tile feeds from there into a per-(tile, bin) partial sum; a second
 * kernel adds each bin's partial sums in tile order.  Only block and grid of
 * the tiling apply to this layout.
 * AZI_LAYOUT_BAND: bins are grouped into bands of R consecutive bins (R =
 * the tiling's band: 4, 8 or 16; other values mean 8) and each band's
 * entries are ordered by pixel id, so the image is read in its own row-major
 * order, a few nearly full cache lines per image row; pieces of tile_nnz
 * entries add into per-bin partial sums that a second kernel adds in order.
 * Images up to 2^27 pixels.
 * AZI_LAYOUT_FUSED (one-dimensional plans, AZI_SPLIT_BBOX or _NONE): no
 * matrix is read per frame.  Each workgroup takes an 8 x 64 image tile,
 * recomputes its pixels' radial extents and bounding-box shares from the
 * plan's geometry with the operations of the plan builder (Sections 3, 4.1;
 * the coefficients are the stored matrix's, bit for bit for the radial
 * units, to rounding where atan / sin enter), and sums every bin
 * of the tile's window into a per-(tile, bin) partial; a second kernel adds
 * each bin's partials in tile order.  With azi_integrate1d_raw the cast and
 * correction happen in the same kernel.  Only the tiling's grid applies.
 * Batches do not take this layout.
 * AZI_LAYOUT_RUN: the band layout with bands of 4 bins, stored per run: the
 * entries of one pixel inside one band (consecutive bins) share one word
 * (pixel, first row, count) and one gather of the pixel; the coefficients
 * follow slot-major per group of 64 runs.  Pieces hold tile_nnz / 2 runs;
 * the band value of the tiling is ignored (bands of 4 bins); block 128
 * gives 128-thread workgroups (for batches of small images), any other
 * value 256.  Images up to 2^27 pixels; a batch up to 2^31 runs and
 * entries.
 * Set before azi_plan_upload (a later call re-uploads).  AZI_ESTATE once
 * corrections are set on an uploaded plan.  A refused or failed call leaves
 * the plan in its previous layout (if the re-upload of the new layout fails,
 * the previous layout is uploaded again; should that fail too, the plan is
 * left off the device, as after a failed azi_plan_upload).
 */
#define AZI_LAYOUT_PIXEL 0
#define AZI_LAYOUT_RING 1
#define AZI_LAYOUT_TILE 2
#define AZI_LAYOUT_BAND 3
#define AZI_LAYOUT_FUSED 4
#define AZI_LAYOUT_RUN 5
int azi_plan_set_layout(azi_plan* plan, int32_t layout);
int azi_plan_get_layout(const azi_plan* plan, int32_t* layout);

/* Place the plan on HIP device `device`: copies the CSR and CSC matrices,
 * the tile schedule and allocates the plan's work buffers.  Synchronous.
 * Errors: AZI_EDEVICE (no such device / HIP failure), AZI_ENOMEM. */
int azi_plan_upload(azi_plan* plan, int32_t device);

/* Device memory held by the plan, in bytes (0 before upload). */
int64_t azi_plan_device_bytes(const azi_plan* plan);

/*
 * Per-pixel correction arrays of Section 6.4 (device pointers of the storage
 * type, npix values each, or NULL for "absent").  The plan keeps a copy of
 * dark and of norm = (flat * solid) * polar, formed once here, so the
 * per-frame map is x = (raw - dark) / norm; with the band or run layout
 * and AZI_STAGE_FUSE it also keeps the (dark, 1 / norm) pairs its gather
 * reads.
 * A float64 plan whose dark values are all exactly floats keeps them as
 * 12-byte records (float dark, double 1 / norm) instead of 16-byte pairs:
 * the results are the same bits, the gather reads 4 bytes less per pixel.
 * Passing all NULL removes the corrections.  Runs on `stream` and
 * synchronises it.  Needs an uploaded plan.
 */
int azi_plan_set_corrections(azi_plan* plan, const void* dark, const void* flat,
                             const void* solid, const void* polar, void* stream);

/* Bytes per pixel of the per-pixel correction the band gather reads (16 or
 * 8 for pairs of float64 / float32, 12 for the records above; with
 * AZI_STAGE_FOLD the dark value alone, stored per run rather than per
 * pixel: 2 for integer counts of 16 bits, 4 as a float, else the storage
 * size), or 0 when the raw-frame
 * path keeps no such array (no corrections or no dark with
 * AZI_STAGE_FOLD, AZI_STAGE_FOLD_SUM with float64 sums, or another layout
 * or stage).  0 for a NULL plan. */
int32_t azi_plan_correction_bytes(const azi_plan* plan);

/*
 * Cast and correction map (Section 6.4): x[p] = (T(raw[p]) - dark[p]) / norm[p]
 * for the npix pixels, in the storage type T, absent corrections acting as
 * identity.  raw (device, raw_dtype one of AZI_I16..AZI_F64), x (device).
 */
int azi_correct(const azi_plan* plan, const void* raw, int32_t raw_dtype, void* x,
                void* stream);

/*
 * Integrate one corrected image (Section 5.2.1): out_I, out_W, out_U (device,
 * npt values of the storage type; out_W / out_U may be NULL) receive I, W, U;
 * a bin with U == 0 gets I = empty.  x (device, npix values of the storage
 * type) is the corrected image (azi_correct), or the raw image itself when no
 * corrections apply.
 */
int azi_integrate1d(const azi_plan* plan, const void* x, void* out_I, void* out_W,
                    void* out_U, double empty, void* stream);

/*
 * The whole per-frame pipeline of Section 6.4 on a raw image: cast and
 * correction (into the plan's layout) in the plan's work image, then the
 * integration.  raw is a device image of raw_dtype.
 */
int azi_integrate1d_raw(const azi_plan* plan, const void* raw, int32_t raw_dtype,
                        void* out_I, void* out_W, void* out_U, double empty,
                        void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * azi_integrate1d_raw with the same kernels, the same order of sums and so
 * the same bits, but the partial sums go to a static device array of
 * azi_noalloc_scratch_bytes() bytes (8 MiB) instead of the plan's own work
 * buffer.  Every device the library runs on holds one such array until the
 * process ends; its address is looked up on the first call on each device.
 * The call allocates nothing and does not synchronise.
 *   Layouts: run and band (stage AZI_STAGE_FUSE, _FOLD or _FOLD_SUM), tile and
 *   fused; the pixel and ring layouts (which also need the plan's work
 *   image) give AZI_EINVAL.
 *   Limit: a plan whose partial sums exceed the array (16 bytes per slot:
 *   4 slots per band piece, one per (tile, bin) of the tile and fused
 *   layouts) gives AZI_EINVAL; at the default tiling a ~1e7-pixel frame
 *   with 3162 bins needs about 0.5 MB.
 *   Sharing: all calls on one device share its array and every call
 *   overwrites what it needs before reading it, so sequential calls, on one
 *   stream or ordered by events, are safe; calls that overlap in time on
 *   one device (different streams or threads) race on it.
 */
int azi_integrate1d_raw_noalloc(const azi_plan* plan, const void* raw, int32_t raw_dtype,
                                void* out_I, void* out_W, void* out_U, double empty,
                                void* stream);
int64_t azi_noalloc_scratch_bytes(void);

/*
 * The two stages of azi_integrate1d_raw as separate calls (for callers that
 * time or overlap them): azi_plan_stage runs the cast and correction of a
 * raw image into the plan's work image, in the plan's layout;
 * azi_integrate1d_staged integrates the work image as it stands.
 */
int azi_plan_stage(const azi_plan* plan, const void* raw, int32_t raw_dtype, void* stream);
int azi_integrate1d_staged(const azi_plan* plan, void* out_I, void* out_W, void* out_U,
                           double empty, void* stream);

/*
 * Adjoint of azi_integrate1d.  Since dI_b/dx_p = A_bp / U_b and
 * dW_b/dx_p = A_bp, the gradient with respect to the corrected image is
 *     gx_p = sum_b A_bp (grad_I[b] / U[b] + grad_W[b])
 * (an empty bin contributes nothing).  U (device, npt) is the forward's U
 * output; grad_I, grad_W (device, npt) may each be NULL (zero).  If wrt_raw
 * is nonzero and corrections are set, gx is further divided by norm, giving
 * the gradient with respect to the raw counts.  grad_x (device, npix).
 */
int azi_integrate1d_backward(const azi_plan* plan, const void* U, const void* grad_I,
                             const void* grad_W, void* grad_x, int32_t wrt_raw,
                             void* stream);

/*
 * Batches: n plans of one storage type, accumulation mode and layout are
 * stacked into one block-diagonal matrix on `device` (Section 5.2.2 notes
 * several detectors handled together).  Images, outputs and gradients of a
 * batch are flat concatenations in plan order; azi_batch_info gives the
 * offsets.  The batch copies the matrices; the plans may be destroyed after.
 */
int azi_batch_create(azi_plan* const* plans, int32_t n, int32_t device, azi_batch** out);
int azi_batch_destroy(azi_batch* batch);

/* Sizes and offsets (host outputs, each may be NULL): pix_off[n + 1] and
 * bin_off[n + 1] are the start of every instance in the flat image and
 * output arrays. */
int azi_batch_info(const azi_batch* batch, int32_t* n, int64_t* npix, int64_t* npt,
                   int64_t* nnz, int64_t* pix_off, int64_t* bin_off);

/* Tiling of a batch (as for plans; a batch starts with its first plan's).
 * Synchronises the device. */
int azi_batch_set_tiling(azi_batch* batch, const azi_tiling* tiling);

/* A batch's tiling and number of tiles (each may be NULL). */
int azi_batch_get_tiling(const azi_batch* batch, azi_tiling* tiling, int32_t* ntiles);

/* Forward of every instance in one launch (plus one small fix-up launch for
 * bins split across tiles): x, out_I, out_W, out_U as in azi_integrate1d,
 * concatenated. */
int azi_batch_forward(azi_batch* batch, const void* x, void* out_I, void* out_W,
                      void* out_U, double empty, void* stream);

/* Forward of raw images (raw_dtype, concatenated): cast into the batch's
 * work image (in its layout), then as azi_batch_forward.  Batches carry no
 * correction arrays. */
int azi_batch_forward_raw(azi_batch* batch, const void* raw, int32_t raw_dtype, void* out_I,
                          void* out_W, void* out_U, double empty, void* stream);

/* The same result computed instance by instance with the single-plan kernels
 * (one launch sequence per instance): the baseline the batch replaces. */
int azi_batch_forward_loop(azi_batch* batch, const void* x, void* out_I, void* out_W,
                           void* out_U, double empty, void* stream);

/* Adjoint of azi_batch_forward (as azi_integrate1d_backward, wrt the
 * corrected images), all instances in one launch sequence. */
int azi_batch_backward(azi_batch* batch, const void* U, const void* grad_I,
                       const void* grad_W, void* grad_x, void* stream);

/*
 * Autotuner: times candidate tilings (tile_nnz, block, variant, grid, band) on the batch's own
 * data with HIP events on `stream`, keeps the fastest (azi_batch_set_tiling)
 * and writes a JSON report of all candidates into report (host, report_len
 * bytes, may be NULL).  x, out_* are device buffers as for azi_batch_forward
 * (their contents are overwritten).  Synchronous.
 */
int azi_batch_autotune(azi_batch* batch, const void* x, void* out_I, void* out_W,
                       void* out_U, void* stream, char* report, int32_t report_len);

/*
 * Autotuner for one plan: times candidate layouts and tilings (run, band
 * and pixel layouts for one-dimensional plans, the pixel layout's load
 * variants and tiles and the run layout for 2-D plans) on the plan's own
 * corrected image x with HIP events on `stream` (azi_integrate1d), keeps the
 * fastest (azi_plan_set_layout / azi_plan_set_tiling) and writes a JSON
 * report into report (host, report_len bytes, may be NULL).  While the plan
 * has corrections, only tilings of its current layout are tried.  x, out_*
 * are device buffers as for azi_integrate1d (their contents are
 * overwritten).  Synchronous; needs an uploaded plan.
 */
int azi_plan_autotune(azi_plan* plan, const void* x, void* out_I, void* out_W, void* out_U,
                      void* stream, char* report, int32_t report_len);

/*
 * Capture a batch's forward (and, when grad_I or grad_W is non-NULL, its
 * backward right after, reading the U written by the forward) into a HIP
 * graph bound to these device buffers.  Replays with azi_graph_launch.
 */
int azi_graph_create_batch(azi_batch* batch, const void* x, void* out_I, void* out_W,
                           void* out_U, double empty, const void* grad_I,
                           const void* grad_W, void* grad_x, void* stream,
                           azi_graph** out);

/* Capture one plan's raw-image pipeline (azi_integrate1d_raw) into a graph. */
int azi_graph_create_plan(const azi_plan* plan, const void* raw, int32_t raw_dtype,
                          void* out_I, void* out_W, void* out_U, double empty,
                          void* stream, azi_graph** out);

/*
 * Replay a captured graph on `stream` (no allocation, no synchronisation),
 * and free one.  A graph records the device addresses of its plan's or
 * batch's matrices and work buffers and of the caller's buffers: it stays
 * valid while all of them do, i.e. until the plan or batch is destroyed,
 * re-uploaded, given another layout, tiling or corrections, or the
 * caller's buffers are freed.  Destroy and capture again after any of
 * these.  azi_graph_launch: AZI_EINVAL for a NULL graph; azi_graph_destroy(NULL)
 * does nothing.
 */
int azi_graph_launch(azi_graph* graph, void* stream);
int azi_graph_destroy(azi_graph* graph);

#ifdef __cplusplus
}
#endif

#endif /* AZINT_H */
