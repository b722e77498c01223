// Device plan builder kernels (one- and two-dimensional plans, Sections
// 3.3, 4.1, 4.2 and 5.2.1): per-pixel extents and entries as the host builder forms
// them, a scan for the pixel-major offsets, and a stable least-significant-
// digit radix sort that turns the pixel-major entry list into the bin-major
// (CSR) order and into the band order of the gather kernels.  Integer sums
// only; no floating-point atomics.
#include "plan_device.h"

#include "pixel_math.h"

namespace azi {
namespace {

constexpr int kB = kBuildBlock;

__global__ void k_extents(azi_geom g, int32_t unit, int32_t split, double* lo, double* hi,
                          double* bmin, double* bmax) {
    __shared__ double smin[kB], smax[kB];
    const int64_t npix = (int64_t)g.h * g.w;
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    double a = HUGE_VAL, b = -HUGE_VAL;
    if (p < npix) {
        const Extent e = pixel_extent(p / g.w, p % g.w, g);
        if (split == AZI_SPLIT_NONE) {
            a = b = to_unit(e.mid, unit, g.dist_m, g.wavelength_m);
            lo[p] = a;
        } else {
            a = to_unit(e.lo, unit, g.dist_m, g.wavelength_m);
            b = to_unit(e.hi, unit, g.dist_m, g.wavelength_m);
            lo[p] = a;
            hi[p] = b;
        }
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    __syncthreads();
    for (int k = kB / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            smin[threadIdx.x] = vmin(smin[threadIdx.x], smin[threadIdx.x + k]);
            smax[threadIdx.x] = vmax(smax[threadIdx.x], smax[threadIdx.x + k]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bmin[blockIdx.x] = smin[0];
        bmax[blockIdx.x] = smax[0];
    }
}

__global__ void k_minmax(const double* bmin, const double* bmax, int64_t n, double* out2) {
    __shared__ double smin[kB], smax[kB];
    double a = HUGE_VAL, b = -HUGE_VAL;
    for (int64_t i = threadIdx.x; i < n; i += kB) {
        a = vmin(a, bmin[i]);
        b = vmax(b, bmax[i]);
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    __syncthreads();
    for (int k = kB / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            smin[threadIdx.x] = vmin(smin[threadIdx.x], smin[threadIdx.x + k]);
            smax[threadIdx.x] = vmax(smax[threadIdx.x], smax[threadIdx.x + k]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = smin[0];
        out2[1] = smax[0];
    }
}

// The entries of pixel p, in ascending bin (row) order, handed to
// emit(bin, c).  nazim > 0: two-dimensional rows (wedge * npt + radial bin),
// npt being the radial bins.
template <class Emit>
__device__ inline void pixel_entries(const azi_geom& g, int32_t unit, int32_t split, int64_t p,
                                     const double* lo, const double* hi, double pmin,
                                     double delta, int32_t npt, int32_t nazim, Emit&& emit) {
    if (nazim > 0) {
        const Grid2d G{pmin, delta, (2.0 * M_PI) / nazim, npt, nazim};
        const int64_t i = p / g.w, j = p % g.w;
        if (split == AZI_SPLIT_BBOX) bbox2d_entries(i, j, g, lo[p], hi[p], G, emit);
        else if (split == AZI_SPLIT_FULL) full2d_entries(i, j, g, unit, lo[p], hi[p], G, emit);
        else none2d_entry(i, j, g, (lo[p] - pmin) / delta, G, emit);
        return;
    }
    if (split == AZI_SPLIT_BBOX) {
        bbox_pixel(lo[p], hi[p], pmin, delta, npt, emit);
    } else if (split == AZI_SPLIT_FULL) {
        full_pixel(p / g.w, p % g.w, g, unit, lo[p], hi[p], pmin, delta, npt, emit);
    } else {
        const double fc = (lo[p] - pmin) / delta;
        if (fc >= 0.0 && fc <= (double)npt) emit(vmin((int32_t)::floor(fc), npt - 1), 1.0);
    }
}

__global__ void k_count(azi_geom g, int32_t unit, int32_t split, const double* lo,
                        const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                        int32_t* count) {
    const int64_t npix = (int64_t)g.h * g.w;
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= npix) return;
    int32_t c = 0;
    pixel_entries(g, unit, split, p, lo, hi, pmin, delta, npt, nazim,
                  [&](int32_t, double) { ++c; });
    count[p] = c;
}

__global__ void k_fill(azi_geom g, int32_t unit, int32_t split, const double* lo,
                       const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                       const int32_t* colptr, int32_t* rowidx, double* cdata, int32_t* pix) {
    const int64_t npix = (int64_t)g.h * g.w;
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= npix) return;
    int64_t k = colptr[p];
    const int64_t k1 = colptr[p + 1];
    pixel_entries(g, unit, split, p, lo, hi, pmin, delta, npt, nazim, [&](int32_t b, double c) {
        if (k < k1) {
            rowidx[k] = b;
            cdata[k] = c;
            pix[k] = (int32_t)p;
        }
        ++k;
    });
}

// ---------------------------------------------------------------------------
// Exclusive scan: tiles of kScanTile counts; per-tile totals, a one-block
// scan of the totals, then each tile re-scanned with its offset.
// ---------------------------------------------------------------------------
constexpr int kScanPer = 8;
constexpr int kScanTile = kB * kScanPer;

// Exclusive scan of one value per thread over the block; returns the
// thread's offset and leaves the block total in *total.
__device__ inline int64_t block_exclusive(int64_t v, int64_t* sh, int64_t* total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = 1; k < kB; k <<= 1) {
        const int64_t add = (int)threadIdx.x >= k ? sh[threadIdx.x - k] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t incl = sh[threadIdx.x];
    *total = sh[kB - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const int32_t* in, int64_t n, int64_t* tile_sum) {
    __shared__ int64_t sh[kB];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t v = 0;
    for (int j = 0; j < kScanPer; ++j)
        if (base + j < n) v += in[base + j];
    int64_t total;
    (void)block_exclusive(v, sh, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void k_scan_top(int64_t* tile_sum, int64_t ntiles, int64_t* total_out) {
    __shared__ int64_t sh[kB];
    int64_t carry = 0;
    for (int64_t c = 0; c < ntiles; c += kB) {
        const int64_t i = c + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        int64_t total;
        const int64_t off = block_exclusive(v, sh, &total);
        if (i < ntiles) tile_sum[i] = carry + off;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_apply(const int32_t* in, int64_t n, const int64_t* tile_off,
                             const int64_t* total, int32_t* out) {
    __shared__ int64_t sh[kB];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int64_t sum = 0;
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        sum += v[j];
    }
    int64_t btotal;
    int64_t run = tile_off[blockIdx.x] + block_exclusive(sum, sh, &btotal);
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < n) out[base + j] = (int32_t)run;
        run += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int32_t)*total;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  A tile of kSortTile keys is read in
// chunks of kB (one key per thread, in order); inside a wavefront the keys
// with the same digit find each other by eight ballots, wavefronts are
// ordered through LDS counts, chunks through running per-digit counts, and
// tiles through the digit-major exclusive scan of the per-tile histograms.
// ---------------------------------------------------------------------------
constexpr int kDigits = 256;
constexpr int kChunks = 16;
constexpr int kSortTile = kB * kChunks;
constexpr int kWaves = kB / 64;

__device__ inline int32_t key_at(const int32_t* keys, int64_t e) { return keys[e]; }

__global__ void k_digit_hist(const int32_t* keys, int64_t n, int shift, int64_t ntiles,
                             int32_t* hist) {
    __shared__ int32_t cnt[kDigits];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kChunks; ++c) {
        const int64_t e = base + (int64_t)c * kB + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(key_at(keys, e) >> shift) & (kDigits - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_digit_scatter(const int32_t* keys_in, const int32_t* vals_in, int64_t n,
                                int shift, int64_t ntiles, const int32_t* offs,
                                int32_t* keys_out, int32_t* vals_out) {
    __shared__ int32_t running[kDigits];
    __shared__ int32_t wc[kWaves][kDigits];
    const int t = threadIdx.x;
    const int wave = t / 64;
    const int lane = t % 64;
    running[t] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kChunks; ++c) {
        for (int w = 0; w < kWaves; ++w) wc[w][t] = 0;
        __syncthreads();
        const int64_t e = base + (int64_t)c * kB + t;
        const bool valid = e < n;
        const int32_t key = valid ? keys_in[e] : 0;
        const int d = (key >> shift) & (kDigits - 1);
        unsigned long long m = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1;
            const unsigned long long b = __ballot(on);
            m &= on ? b : ~b;
        }
        const unsigned long long below = lane ? (m & (~0ull >> (64 - lane))) : 0ull;
        const int rank = __popcll(below);
        if (valid && (63 - __clzll(m)) == lane) wc[wave][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int32_t before = running[d];
            for (int w = 0; w < wave; ++w) before += wc[w][d];
            const int64_t pos = (int64_t)offs[(int64_t)d * ntiles + blockIdx.x] + before + rank;
            keys_out[pos] = key;
            vals_out[pos] = vals_in ? vals_in[e] : (int32_t)e;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += wc[w][t];
        running[t] += add;
        __syncthreads();
    }
}

__global__ void k_div(const int32_t* rowidx, int64_t n, int32_t R, int32_t* key) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) key[i] = rowidx[i] / R;
}

__global__ void k_bounds(const int32_t* sorted, int64_t n, int32_t nrows, int32_t* indptr) {
    const int64_t b = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (b > nrows) return;
    int64_t lo = 0, hi = n;  // first position with key >= b
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (sorted[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    indptr[b] = (int32_t)lo;
}

template <class T>
__global__ void k_gather(const int32_t* perm, int64_t n, int64_t n_alloc, const int32_t* pix,
                         const double* cdata, int32_t* indices, T* data, double* data64) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n_alloc) return;
    if (i < n) {
        const int32_t k = perm[i];
        const double c = cdata[k];
        indices[i] = pix[k];
        data[i] = (T)c;
        if (data64) data64[i] = c;
    } else {
        indices[i] = 0;
        data[i] = (T)0;
    }
}

template <class T>
__global__ void k_band_entries(const int32_t* perm, int64_t n, int64_t n_alloc,
                               const int32_t* rowidx, const int32_t* pix, const double* cdata,
                               int32_t R, int32_t* packed, T* coef) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n_alloc) return;
    if (i < n) {
        const int32_t k = perm[i];
        packed[i] = ((rowidx[k] % R) << kBandShift) | pix[k];
        coef[i] = (T)cdata[k];
    } else {
        packed[i] = 0;
        coef[i] = (T)0;
    }
}

template <class T>
__global__ void k_to_storage(const double* in, int64_t n, T* out) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) out[i] = (T)in[i];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

bool grid_fits(int64_t n) { return (n + kB - 1) / kB <= (int64_t)INT32_MAX; }

}  // namespace

hipError_t launch_extents(const azi_geom& g, int32_t unit, int32_t split, double* lo, double* hi,
                          double* bmin, double* bmax, hipStream_t s) {
    const int64_t npix = (int64_t)g.h * g.w;
    if (!grid_fits(npix)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_extents, dim3(blocks_for(npix)), dim3(kB), 0, s, g, unit, split, lo, hi,
                       bmin, bmax);
    return hipGetLastError();
}

hipError_t launch_minmax(const double* bmin, const double* bmax, int64_t n, double* out2,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kB), 0, s, bmin, bmax, n, out2);
    return hipGetLastError();
}

hipError_t launch_count(const azi_geom& g, int32_t unit, int32_t split, const double* lo,
                        const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                        int32_t* count, hipStream_t s) {
    const int64_t npix = (int64_t)g.h * g.w;
    if (!grid_fits(npix)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_count, dim3(blocks_for(npix)), dim3(kB), 0, s, g, unit, split, lo, hi,
                       pmin, delta, npt, nazim, count);
    return hipGetLastError();
}

hipError_t launch_fill(const azi_geom& g, int32_t unit, int32_t split, const double* lo,
                       const double* hi, double pmin, double delta, int32_t npt, int32_t nazim,
                       const int32_t* colptr, int32_t* rowidx, double* cdata, int32_t* pix,
                       hipStream_t s) {
    const int64_t npix = (int64_t)g.h * g.w;
    if (!grid_fits(npix)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(npix)), dim3(kB), 0, s, g, unit, split, lo, hi,
                       pmin, delta, npt, nazim, colptr, rowidx, cdata, pix);
    return hipGetLastError();
}

size_t scan_work_bytes(int64_t n) {
    const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    return (size_t)(ntiles + 1) * sizeof(int64_t);
}

hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int64_t* total, void* work,
                       hipStream_t s) {
    const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    int64_t* tile_sum = static_cast<int64_t*>(work);
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kB), 0, s, in, n, tile_sum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kB), 0, s, tile_sum, ntiles, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)std::max<int64_t>(ntiles, 1)), dim3(kB), 0, s,
                       in, n, tile_sum, total, out);
    return hipGetLastError();
}

size_t sort_work_bytes(int64_t n) {
    const int64_t ntiles = std::max<int64_t>((n + kSortTile - 1) / kSortTile, 1);
    const int64_t nh = ntiles * kDigits;
    // ping-pong keys and values, histograms, offsets (+ total), scan work
    return (size_t)(2 * n * 4 + nh * 4 + (nh + 1) * 4 + 8) + scan_work_bytes(nh) + 256;
}

hipError_t launch_sort(const int32_t* keys, int64_t n, int bits, int32_t* keys_out,
                       int32_t* vals_out, void* work, hipStream_t s) {
    const int64_t ntiles = std::max<int64_t>((n + kSortTile - 1) / kSortTile, 1);
    if (ntiles > (int64_t)INT32_MAX || n >= (int64_t)INT32_MAX) return hipErrorInvalidValue;
    const int64_t nh = ntiles * kDigits;
    char* w = static_cast<char*>(work);
    int32_t* kb = reinterpret_cast<int32_t*>(w);
    int32_t* vb = kb + n;
    int32_t* hist = vb + n;
    int32_t* offs = hist + nh;
    int64_t* total = reinterpret_cast<int64_t*>(
        (reinterpret_cast<uintptr_t>(offs + nh + 1) + 7) & ~(uintptr_t)7);
    void* scan_work = reinterpret_cast<void*>(
        (reinterpret_cast<uintptr_t>(total + 1) + 15) & ~(uintptr_t)15);
    const int passes = std::max(1, (bits + 7) / 8);
    // pass k reads (kin, vin) and writes (kout, vout); the last pass writes
    // the caller's buffers
    const int32_t* kin = keys;
    const int32_t* vin = nullptr;
    for (int pass = 0; pass < passes; ++pass) {
        const bool last = pass + 1 == passes;
        // alternate so that the last pass lands in the caller's buffers
        const bool to_caller = ((passes - 1 - pass) % 2) == 0;
        int32_t* kout = to_caller ? keys_out : kb;
        int32_t* vout = to_caller ? vals_out : vb;
        (void)last;
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)ntiles), dim3(kB), 0, s, kin, n, shift,
                           ntiles, hist);
        hipError_t e = launch_scan(hist, nh, offs, total, scan_work, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)ntiles), dim3(kB), 0, s, kin, vin, n,
                           shift, ntiles, offs, kout, vout);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        kin = kout;
        vin = vout;
    }
    return hipSuccess;
}

hipError_t launch_div(const int32_t* rowidx, int64_t n, int32_t R, int32_t* key, hipStream_t s) {
    if (!grid_fits(n)) return hipErrorInvalidValue;
    if (n > 0) hipLaunchKernelGGL(k_div, dim3(blocks_for(n)), dim3(kB), 0, s, rowidx, n, R, key);
    return hipGetLastError();
}

hipError_t launch_bounds(const int32_t* sorted, int64_t n, int32_t nrows, int32_t* indptr,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_bounds, dim3(blocks_for((int64_t)nrows + 1)), dim3(kB), 0, s, sorted, n,
                       nrows, indptr);
    return hipGetLastError();
}

hipError_t launch_gather(const int32_t* perm, int64_t n, int64_t n_alloc, const int32_t* pix,
                         const double* cdata, int32_t* indices, void* data, int32_t dtype,
                         double* data64, hipStream_t s) {
    if (!grid_fits(n_alloc)) return hipErrorInvalidValue;
    if (dtype == AZI_F64)
        hipLaunchKernelGGL(k_gather<double>, dim3(blocks_for(n_alloc)), dim3(kB), 0, s, perm, n,
                           n_alloc, pix, cdata, indices, static_cast<double*>(data), data64);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(blocks_for(n_alloc)), dim3(kB), 0, s, perm, n,
                           n_alloc, pix, cdata, indices, static_cast<float*>(data), data64);
    return hipGetLastError();
}

hipError_t launch_band_entries(const int32_t* perm, int64_t n, int64_t n_alloc,
                               const int32_t* rowidx, const int32_t* pix, const double* cdata,
                               int32_t R, int32_t* packed, void* coef, int32_t dtype,
                               hipStream_t s) {
    if (!grid_fits(n_alloc)) return hipErrorInvalidValue;
    if (dtype == AZI_F64)
        hipLaunchKernelGGL(k_band_entries<double>, dim3(blocks_for(n_alloc)), dim3(kB), 0, s,
                           perm, n, n_alloc, rowidx, pix, cdata, R, packed,
                           static_cast<double*>(coef));
    else
        hipLaunchKernelGGL(k_band_entries<float>, dim3(blocks_for(n_alloc)), dim3(kB), 0, s,
                           perm, n, n_alloc, rowidx, pix, cdata, R, packed,
                           static_cast<float*>(coef));
    return hipGetLastError();
}

hipError_t launch_to_storage(const double* in, int64_t n, void* out, int32_t dtype,
                             hipStream_t s) {
    if (!grid_fits(n)) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    if (dtype == AZI_F64)
        hipLaunchKernelGGL(k_to_storage<double>, dim3(blocks_for(n)), dim3(kB), 0, s, in, n,
                           static_cast<double*>(out));
    else
        hipLaunchKernelGGL(k_to_storage<float>, dim3(blocks_for(n)), dim3(kB), 0, s, in, n,
                           static_cast<float*>(out));
    return hipGetLastError();
}

}  // namespace azi
