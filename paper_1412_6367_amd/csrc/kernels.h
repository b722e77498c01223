// Launch wrappers of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace azi {

struct ForwardLaunch {
    const Tile* tiles = nullptr;
    int32_t ntiles = 0;
    const Split* splits = nullptr;
    int32_t nsplits = 0;
    const int32_t* rowptr = nullptr;   // concatenated row pointers (global nnz positions)
    const int32_t* indices = nullptr;  // pixel ids (global)
    const void* data = nullptr;        // coefficients, storage type
    const void* x = nullptr;           // corrected image(s), storage type
    void* I = nullptr;
    void* W = nullptr;                 // may be null
    void* U = nullptr;                 // may be null
    void* parts = nullptr;             // partial sums of split rows (16 bytes each)
    double empty = 0.0;
    int32_t block = 256;
    int32_t variant = 2;               // load layout / unroll / streaming, see kVariants
    int32_t grid = 0;                  // 0: one workgroup per tile
    int32_t dtype = AZI_F64;
    int32_t accum = AZI_ACC_F64;
};

constexpr int32_t kNumVariants = AZI_NUM_VARIANTS;

hipError_t launch_forward(const ForwardLaunch& a, hipStream_t s);

struct BackwardLaunch {
    const int32_t* colptr = nullptr;   // npix + 1 (global nnz positions)
    const int32_t* rowidx = nullptr;   // global bin ids
    const int32_t* first = nullptr;    // when set: each pixel's bins are consecutive from
                                       // first[p] (rowidx then unused); cdata and v
                                       // then hold 4 spare elements past their end
    const void* cdata = nullptr;       // storage type
    const void* U = nullptr;           // forward U, storage type
    const void* gI = nullptr;          // may be null
    const void* gW = nullptr;          // may be null
    const void* norm = nullptr;        // divide the result by it when non-null
    double* v = nullptr;               // work buffer, npt (+ 4 spare) doubles
    void* gx = nullptr;                // npix, storage type
    int64_t npix = 0;
    int64_t npt = 0;
    int32_t dtype = AZI_F64;
};

hipError_t launch_backward(const BackwardLaunch& a, hipStream_t s);

// x[i] = (T(raw[order ? order[i] : i]) - dark[i]) / norm[i] for i < n (order,
// dark, norm may be null).  With `order`, this is also the plain permutation
// (cast) of an image into ring positions.
hipError_t launch_correct(const void* raw, int32_t raw_dtype, const int32_t* order,
                          const void* dark, const void* norm, void* x, int32_t dtype,
                          int64_t n, hipStream_t s);

// Per-pixel correction of the raw-frame band gather: (dark, 1 / norm) as a
// pair of the storage type, or, for float64 plans whose dark values are all
// floats, as a 12-byte record (4 bytes less per pixel, same results).  With
// the normalisation folded into the coefficients (AZI_STAGE_FOLD, run
// layout) dark alone is subtracted, stored once per run beside the run
// words and read with them (run z's value is the dark of its pixel), which
// leaves the raw count as the only gather: as uint16 when every dark value
// is an integer in [0, 65535] (kCorrRunDarkU16), as float for float64 plans
// whose dark values are all floats (kCorrRunDarkF32), else in the storage
// type (kCorrRunDark); the conversions are exact, so all give the same bits.
constexpr int32_t kCorrPair = 0, kCorrRecord12 = 1, kCorrRunDarkF32 = 2, kCorrRunDark = 3,
                  kCorrRunDarkU16 = 4;
// Element type of a run-indexed dark array.
template <class V>
struct RunDark {
    V v;
};
struct Corr12 {
    float dark;
    uint32_t inv_lo, inv_hi;  // the two halves of the double 1 / norm
};
static_assert(sizeof(Corr12) == 12, "12-byte correction record");

// Band integration: k_band over pieces [0, npieces) fills the partial slots,
// then k_band_reduce finishes bins [b0, b1).  x is the corrected image.
struct BandLaunch {
    const BandPiece* pieces = nullptr;
    int32_t npieces = 0;
    const int32_t* packed = nullptr;   // entries, or the runs when gbase is set
    const int32_t* gbase = nullptr;    // run encoding (R = kRunRows): group coefficient bases
    const void* coef = nullptr;
    const int32_t* bin_slot = nullptr;
    const int32_t* bin_count = nullptr;
    int32_t max_count = INT32_MAX;     // largest bin_count (selects the reduction form)
    int32_t R = 8;
    // run encoding: 1 = one band per workgroup (the pieces are BandPiece
    // per piece); 4 or 8 = that many neighbouring bands per workgroup (the
    // pieces hold `waves` entries per workgroup, see k_runs_grouped)
    int32_t waves = 1;
    int64_t b0 = 0, b1 = 0;
    const void* x = nullptr;
    // raw-frame form: when `raw` is set, x is ignored and each gathered pixel
    // is (T(raw) - corr.x) * corr.y with corr the (dark, 1 / norm) pairs of
    // launch_corr_pair, or just T(raw) when corr is null; 256 threads
    const void* raw = nullptr;
    int32_t raw_dtype = AZI_I32;
    const void* corr = nullptr;
    int32_t corr_kind = kCorrPair;     // kCorrRecord12: Corr12 records (float64 only)
    void* parts = nullptr;
    void* I = nullptr;
    void* W = nullptr;
    void* U = nullptr;
    double empty = 0.0;
    int32_t block = 256;
    int32_t grid = 0;
    int32_t dtype = AZI_F64;
    int32_t accum = AZI_ACC_F64;
    // U of a plan does not depend on the image.  ufix_out: the reduction
    // writes each bin's U (as the accumulator holds it, in double) there and
    // nothing else; ufix_in: the reduction takes U from it instead of from
    // the partial sums (used when the coefficients carry the normalisation,
    // whose sums are then not U).
    double* ufix_out = nullptr;
    const double* ufix_in = nullptr;
    // The frame-independent dark term of W (AZI_STAGE_FOLD_SUM).  wfix_out:
    // the reduction writes each bin's W (as the accumulator holds it, in
    // double) there and nothing else; wsub_in (with ufix_in): the reduction
    // subtracts it from each bin's W before forming I.
    double* wfix_out = nullptr;
    const double* wsub_in = nullptr;
};

hipError_t launch_band(const BandLaunch& a, hipStream_t s);

// Workgroups of the co-scheduled run kernel (`waves` bands; the storage type
// and accumulator of `dtype` / `accum`) that one CU of the current device
// keeps resident, from the runtime's occupancy calculator for the kernel's
// raw-frame, folded-correction form (W accumulated alone; its other forms
// are held to the same 8 wavefronts per SIMD); 0 if the runtime cannot tell.
int32_t runs_resident_per_cu(int32_t dtype, int32_t accum, int32_t waves);

// pair[i] = (dark[i], 1 / norm[i]) in the storage type (0 and 1 where the
// array is null): the per-pixel correction of the fused band gather.
hipError_t launch_corr_pair(const void* dark, const void* norm, void* pair, int32_t dtype,
                            int64_t n, hipStream_t s);
// *flag (device int32) = 1 if some dark[i] is not exactly a float, else 0.
hipError_t launch_dark_is_float(const double* dark, int64_t n, int32_t* flag, hipStream_t s);
// rec[i] = Corr12{(float)dark[i], 1 / norm[i] or 1}; dark must be non-null
// and hold floats only (launch_dark_is_float).
hipError_t launch_corr_record12(const double* dark, const double* norm, void* rec, int64_t n,
                                hipStream_t s);

// Blocked (image-tile) integration: k_block over tiles [0, ntiles) fills the
// partial slots, then k_block_reduce finishes bins [b0, b1).  `img` is the
// raw (img_dtype) or corrected image; dark / norm (storage type, row-major,
// nullable) are applied on the fly.
struct BlockLaunch {
    const BlockTile* tiles = nullptr;
    int32_t ntiles = 0;
    const BlockRow* rows = nullptr;
    const uint16_t* lp = nullptr;
    const void* coef = nullptr;
    const int32_t* bin_ptr = nullptr;
    int64_t b0 = 0, b1 = 0;
    const void* img = nullptr;
    int32_t img_dtype = AZI_F64;
    const void* dark = nullptr;
    const void* norm = nullptr;
    void* parts = nullptr;
    void* I = nullptr;
    void* W = nullptr;
    void* U = nullptr;
    double empty = 0.0;
    int32_t block = 256;
    int32_t grid = 0;
    int32_t dtype = AZI_F64;
    int32_t accum = AZI_ACC_F64;
};

hipError_t launch_block(const BlockLaunch& a, hipStream_t s);

// Moving a raw image into ring positions (with cast and correction):
//   gather   x[q] = f(raw[order[q]]), q in [p0, p1); dark / norm in ring order,
//            `raw` and `order` already offset to the range's start
//   scatter  x[pos[p]] = f(raw[p]), p in [p0, p1); dark / norm row-major
//   tile     the stage tiles [0, ntiles) through LDS; dark / norm row-major
constexpr int32_t kStageGather = 0, kStageScatter = 1, kStageTile = 2;
struct StageLaunch {
    int32_t mode = kStageTile;
    const void* raw = nullptr;
    int32_t raw_dtype = AZI_I32;
    const int32_t* order = nullptr;
    const int32_t* pos = nullptr;
    const StageTile* tiles = nullptr;
    int32_t ntiles = 0;
    const uint16_t* lidx = nullptr;
    const int32_t* dest = nullptr;
    const void* dark = nullptr;
    const void* norm = nullptr;
    void* x = nullptr;
    int32_t dtype = AZI_F64;
    int64_t p0 = 0, p1 = 0;
};

hipError_t launch_stage(const StageLaunch& a, hipStream_t s);

// norm = (flat * solid) * polar over the present arrays; returns false in
// *any when all three are null (norm untouched).
hipError_t launch_norm(const void* flat, const void* solid, const void* polar,
                       void* norm, int32_t dtype, int64_t n, hipStream_t s);

}  // namespace azi
