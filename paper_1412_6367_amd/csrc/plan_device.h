// Device plan builder: launch wrappers (host side).  The builder forms the
// same one- or two-dimensional matrix as the host builder -- per-pixel extents,
// per-pixel entries in pixel-major order, then the bin-major order by a
// stable sort on the bin -- with every bin decision taken by the same IEEE
// operations (pixel_math.h, both sides compiled without contraction).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace azi {

// Per-pixel extents in the output unit: boxes (bbox / full split) give
// lo/hi, no split gives the pixel midpoint in lo.  bmin / bmax receive one
// min / max per block of kBuildBlock pixels (lo and hi resp. midpoint).
constexpr int kBuildBlock = 256;
hipError_t launch_extents(const azi_geom& g, int32_t unit, int32_t split, double* lo, double* hi,
                          double* bmin, double* bmax, hipStream_t s);
// out2 = {min of bmin, max of bmax} over n blocks.
hipError_t launch_minmax(const double* bmin, const double* bmax, int64_t n, double* out2,
                         hipStream_t s);
// Entries per pixel.  npt radial bins; nazim > 0 builds the
// two-dimensional rows (wedge * npt + radial bin) of nazim wedges.
hipError_t launch_count(const azi_geom& g, int32_t unit, int32_t split, const double* lo,
                        const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                        int32_t* count, hipStream_t s);
// Pixel-major entries: rowidx (bin), cdata (coefficient), pix (pixel id) at
// colptr[p] .. colptr[p + 1].
hipError_t launch_fill(const azi_geom& g, int32_t unit, int32_t split, const double* lo,
                       const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                       const int32_t* colptr, int32_t* rowidx, double* cdata, int32_t* pix,
                       hipStream_t s);

// Exclusive scan of n int32 counts into out[0 .. n] (out[n] = total), the
// total also in *total (device int64).  `work` holds scan_work_bytes(n).
size_t scan_work_bytes(int64_t n);
hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int64_t* total, void* work,
                       hipStream_t s);

// Stable sort of the indices 0..n-1 by key[i] >> 0 in [0, 2^bits): vals_out
// receives the sorted indices, keys_out the sorted keys.  `work` holds
// sort_work_bytes(n) bytes.
size_t sort_work_bytes(int64_t n);
hipError_t launch_sort(const int32_t* keys, int64_t n, int bits, int32_t* keys_out,
                       int32_t* vals_out, void* work, hipStream_t s);

// key[k] = rowidx[k] / R.
hipError_t launch_div(const int32_t* rowidx, int64_t n, int32_t R, int32_t* key, hipStream_t s);
// indptr[b] = first position of key >= b in the sorted keys, b = 0 .. nrows.
hipError_t launch_bounds(const int32_t* sorted, int64_t n, int32_t nrows, int32_t* indptr,
                         hipStream_t s);
// Bin-major arrays from the permutation: indices[i] = pix[perm[i]],
// data[i] = cdata[perm[i]] in the storage type (and in double to data64
// when non-null); the padding [n, n_alloc) is zeroed.
hipError_t launch_gather(const int32_t* perm, int64_t n, int64_t n_alloc, const int32_t* pix,
                         const double* cdata, int32_t* indices, void* data, int32_t dtype,
                         double* data64, hipStream_t s);
// Band entries from the permutation by band: packed[i] = (rowidx % R) << 27
// | pix, coef[i] = cdata in the storage type; padding zeroed.
hipError_t launch_band_entries(const int32_t* perm, int64_t n, int64_t n_alloc,
                               const int32_t* rowidx, const int32_t* pix, const double* cdata,
                               int32_t R, int32_t* packed, void* coef, int32_t dtype,
                               hipStream_t s);
// Storage copy of double values (float or double).
hipError_t launch_to_storage(const double* in, int64_t n, void* out, int32_t dtype,
                             hipStream_t s);

}  // namespace azi
