// C ABI of the azimuthal-integration library (declared in include/azint.h):
// plan, batch and graph objects, device placement, argument checking and the
// per-frame entry points, which only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "plan_device.h"
#include "fused.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(AZI_EDEVICE, m);
}

#define AZI_HIP(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Device allocation owned by a plan or batch.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int device = -1;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            if (cur != device) (void)hipSetDevice(device);
            (void)hipFree(p);
            if (cur != device && cur >= 0) (void)hipSetDevice(cur);
        }
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t n, int dev) {
        release();
        device = dev;
        if (n == 0) n = 256;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
    hipError_t upload(const void* src, size_t n, int dev) {
        hipError_t e = alloc(n, dev);
        if (e != hipSuccess || n == 0) return e;
        return hipMemcpy(p, src, n, hipMemcpyHostToDevice);
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Makes `dev` current for the lifetime of the guard, restoring the caller's.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) {
            err = hipSetDevice(dev);
            changed = (err == hipSuccess);
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

constexpr int64_t kPad = 64;  // nonzero arrays: instance starts on 64, 64 spare at the end
// The adjoint reads each pixel's first four coefficients and bin values
// with two vector loads whatever the pixel's count: its coefficient array
// and bin-value vector keep this many spare elements at the end.
constexpr int64_t kAdjPad = 4;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

size_t elem_size(int32_t dtype) { return dtype == AZI_F64 ? 8 : 4; }

size_t elem_size_any(int32_t dtype) {
    switch (dtype) {
        case AZI_I16: case AZI_U16: return 2;
        case AZI_F64: return 8;
        default: return 4;
    }
}

const char* kTilingRule =
    "tiling: tile_nnz 0 or a multiple of 64 in [64, 16384], block one of 64/128/256/512, variant "
    "in [0, AZI_NUM_VARIANTS), grid >= 0, band >= 0, stage one of AZI_STAGE_*";

bool valid_tiling(const azi_tiling& t) {
    return (t.tile_nnz == 0 || (t.tile_nnz >= 64 && t.tile_nnz <= 16384 && t.tile_nnz % 64 == 0)) &&
           (t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512) &&
           t.variant >= 0 && t.variant < azi::kNumVariants && t.grid >= 0 && t.band >= 0 &&
           t.stage >= AZI_STAGE_GATHER && t.stage <= AZI_STAGE_FOLD_SUM;
}

// Below ~4e6 nonzeros (a ~1e6-pixel frame) there are too few 4096-entry
// pieces to fill 256 CUs: 2048 entries (18 us against 21 us at 1e6 pixels).
constexpr int64_t kSmallNnz = (int64_t)1 << 22;

// Nonzeros per piece of a tiling over `nnz` nonzeros: tile_nnz, or for a
// tiling sized by the library (tile_nnz 0) 2048 below kSmallNnz and 4096
// above wherever the pieces are not sized from the device.
// (Batches size each instance's pieces by its own nonzeros, as its plan
// would; the co-scheduled run bands of a batch take these fixed pieces too,
// the rounds of a balanced tiling being those of one plan's launch.)
int32_t piece_nnz(const azi_tiling& t, int64_t nnz) {
    return t.tile_nnz > 0 ? t.tile_nnz : nnz < kSmallNnz ? 2048 : 4096;
}

// Workgroups of one round of a balanced tiling (tile_nnz 0) of a plan's
// co-scheduled run bands: as many as the device keeps resident at once
// (CUs times the run kernel's resident workgroups per CU, from the
// runtime: 8 of 4 wavefronts at its 64 VGPRs or fewer; a round sized for
// more than fit spills a few workgroups into a second round, which costs
// as much as the round itself).  The schedule is cut into the fewest such rounds that keep a
// band's stretch within 2048 runs, each workgroup taking as nearly the same
// work as the bands allow (the ~1e7-pixel frame: one round; 2048^2, 4096^2
// and off-centre frames: 27-36 % faster than pieces of 2048 runs but for
// 4096^2, two rounds, 10 %).  None for the other layouts (0).  Without a
// device, MI355X's 256 CUs at 8 workgroups of 4 wavefronts.
int64_t balanced_tiles(const azi_tiling& t, int device, int32_t waves, int32_t dtype,
                       int32_t accum) {
    if (t.tile_nnz != 0 || waves <= 1) return 0;
    int ncu = 256;
    int32_t per_cu = 32 / waves;
    if (device >= 0) {
        DeviceGuard g(device);
        if (g.err == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) ==
                hipSuccess) {
            const int32_t r = azi::runs_resident_per_cu(dtype, accum, waves);
            if (r > 0) per_cu = r;
        } else {
            ncu = 256;
        }
    }
    return (int64_t)ncu * per_cu;
}

// Stages whose raw-frame path corrects each pixel in the band gather.
bool gather_corrects(int32_t stage) {
    return stage == AZI_STAGE_FUSE || stage == AZI_STAGE_FOLD || stage == AZI_STAGE_FOLD_SUM;
}

// Stages that fold 1 / norm into the coefficients (run layout).
bool folds(int32_t stage) { return stage == AZI_STAGE_FOLD || stage == AZI_STAGE_FOLD_SUM; }

// Fastest measured on the ~1e7-pixel, 3162-bin workload: run layout with
// four neighbouring bands of 4 bins per workgroup, the pieces sized by the
// library (balanced rounds of resident workgroups), raw frames corrected in
// the gather with 1 / norm folded into the coefficients and the dark term
// summed once per correction set (float64: 85 / 88 us warm / flushed with a
// dark value stored per run, against 86 / 89 us for pieces of 2048 runs and
// 106 / 116 us with one band per workgroup and the (dark, 1 / norm) pair
// gathered per pixel).  The workgroup stays at 256 threads,
// the raw-frame band kernel's, so the raw and corrected-image entry points
// sum in the same order.
constexpr azi_tiling kDefaultTiling = {0, 256, 5, 0, 16, AZI_STAGE_FOLD_SUM};
constexpr azi_tiling kDefaultTiling32 = {0, 256, 5, 0, 16, AZI_STAGE_FOLD_SUM};
// Two-dimensional plans (short rows, CSR layout): lane-strided loads of
// whole rows, 4 deep, all through the caches (70 us back to back, 82 us
// after a 1 GiB read-only flush for 1000 x 360 bins of a ~1e7-pixel frame;
// 70 / 86 us with the coefficients non-temporal and 8 deep).
constexpr azi_tiling kDefaultTiling2d = {4096, 256, 1, 0, 1, AZI_STAGE_GATHER};

// Converts double coefficients to the storage type into a padded buffer.
std::vector<char> to_storage(const double* src, int64_t n, int64_t n_alloc, int32_t dtype) {
    std::vector<char> out((size_t)n_alloc * elem_size(dtype), 0);
    if (dtype == AZI_F64) {
        std::memcpy(out.data(), src, (size_t)n * 8);
    } else {
        float* f = reinterpret_cast<float*>(out.data());
        for (int64_t k = 0; k < n; ++k) f[k] = (float)src[k];
    }
    return out;
}

// First bin of every pixel when each pixel's entries lie in consecutive
// bins (every one-dimensional matrix the builder makes); empty otherwise.
// The adjoint then reads one word per pixel instead of one per entry.
std::vector<int32_t> consecutive_first(const azi::HostMatrix& m) {
    std::vector<int32_t> first((size_t)m.npix, 0);
    for (int64_t p = 0; p < m.npix; ++p) {
        const int32_t k0 = m.colptr[p], k1 = m.colptr[p + 1];
        if (k0 == k1) continue;
        first[p] = m.rowidx[k0];
        for (int32_t k = k0 + 1; k < k1; ++k)
            if (m.rowidx[k] != m.rowidx[k0] + (k - k0)) return {};
    }
    return first;
}

// Uploads consecutive_first(m) to buf, or releases buf when the matrix has
// a pixel with non-consecutive bins.
int upload_first(const azi::HostMatrix& m, int device, DevBuf& buf) {
    buf.release();
    if (m.two_d) return AZI_OK;
    std::vector<int32_t> first = consecutive_first(m);
    if (first.empty() && m.npix > 0) return AZI_OK;
    AZI_HIP(buf.upload(first.data(), first.size() * 4, device), "first bins");
    return AZI_OK;
}

}  // namespace

struct azi_plan {
    azi::HostMatrix m;
    azi_geom geom{};
    int32_t dtype = AZI_F64, accum = AZI_ACC_F64, unit = 0, split = AZI_SPLIT_BBOX;
    azi_tiling tiling = kDefaultTiling;
    int32_t layout = AZI_LAYOUT_BAND;
    int device = -1;
    int64_t used = 0;  // ring layout: pixels feeding at least one bin
    DevBuf rowptr, indices, data, colptr, rowidx, cdata, tiles, splits, parts, dark, norm, xwork,
        vwork, order, dark_r, norm_r, pos, stiles, lidx, dest, btiles, brows, blp, bcoef, bin_ptr,
        bparts, npieces_buf, npacked, ncoef, bin_slot, bin_count, nparts_buf, ftiles, fslots,
        fbin_ptr, fparts, corr, cfirst, rgbase, fcoef, ufix, wdark;
    int32_t nstiles = 0, nbtiles = 0, npieces = 0, band_rows = 8, nftiles = 0;
    bool folded = false;  // run layout, AZI_STAGE_FOLD(_SUM), corrections set
    int32_t max_count = INT32_MAX;  // largest number of band partials of a bin
    int32_t corr_kind = azi::kCorrPair;
    int32_t ntiles = 0, nsplits = 0, nparts = 0;
    bool has_dark = false, has_norm = false;
};

struct azi_batch {
    int32_t n = 0, dtype = AZI_F64, accum = AZI_ACC_F64;
    int device = -1;
    int64_t npix = 0, npt = 0, nnz = 0, nnz_alloc = 0;
    std::vector<int64_t> pix_off, bin_off, nz_off, ip_off, tile_off, split_off;
    std::vector<int32_t> rp_host;  // concatenated row pointers, global nnz positions
    azi_tiling tiling = kDefaultTiling;
    int32_t layout = AZI_LAYOUT_BAND;
    int32_t ntiles = 0, nsplits = 0, nparts = 0;
    DevBuf rp, indices, data, colptr, rowidx, cdata, tiles, splits, parts, vwork, order, xwork, pos,
        stiles, lidx, dest, btiles, brows, blp, bcoef, bin_ptr, bparts, npieces_buf, npacked, ncoef,
        bin_slot, bin_count, nparts_buf, cfirst, rgbase;
    int32_t nbtiles = 0, npieces = 0, band_rows = 8;
    int32_t max_count = INT32_MAX;  // largest number of band partials of a bin
    std::vector<int64_t> cz_off;     // CSC entries of instance k
    std::vector<int64_t> piece_off;  // band pieces of instance k
    std::vector<int64_t> btile_off;  // blocked tiles of instance k
    std::vector<int64_t> stile_off;  // stage tiles of instance k: [stile_off[k], stile_off[k+1])
};

struct azi_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = -1;
};

namespace {
int batch_build_bands(azi_batch* b, const std::vector<const azi::HostMatrix*>& ms);
int batch_rebuild_bands(azi_batch* b);
}  // namespace

namespace {

// (Re)builds and uploads the tile schedule of a plan.
int plan_upload_tiles(azi_plan* p) {
    std::vector<azi::Tile> tiles;
    std::vector<azi::Split> splits;
    int32_t nparts = 0;
    azi::build_tiles(p->m.indptr.data(), p->m.npt, 0, 0, 0, piece_nnz(p->tiling, p->m.nnz()),
                     p->tiling.band,
                     tiles, splits, nparts);
    AZI_HIP(p->tiles.upload(tiles.data(), tiles.size() * sizeof(azi::Tile), p->device), "tiles");
    AZI_HIP(p->splits.upload(splits.data(), splits.size() * sizeof(azi::Split), p->device),
            "splits");
    AZI_HIP(p->parts.alloc((size_t)std::max(nparts, 1) * 16, p->device), "partials");
    p->ntiles = (int32_t)tiles.size();
    p->nsplits = (int32_t)splits.size();
    p->nparts = nparts;
    return AZI_OK;
}

int batch_upload_tiles(azi_batch* b, const std::vector<const int32_t*>& indptrs,
                       const std::vector<int32_t>& npts) {
    std::vector<azi::Tile> tiles;
    std::vector<azi::Split> splits;
    int32_t nparts = 0;
    b->tile_off.assign(b->n + 1, 0);
    b->split_off.assign(b->n + 1, 0);
    for (int32_t k = 0; k < b->n; ++k) {
        b->tile_off[k] = (int64_t)tiles.size();
        b->split_off[k] = (int64_t)splits.size();
        const int64_t nnz_k = (int64_t)indptrs[k][npts[k]] - indptrs[k][0];
        azi::build_tiles(indptrs[k], npts[k], b->nz_off[k], b->bin_off[k], b->ip_off[k],
                         piece_nnz(b->tiling, nnz_k), b->tiling.band, tiles, splits, nparts);
    }
    b->tile_off[b->n] = (int64_t)tiles.size();
    b->split_off[b->n] = (int64_t)splits.size();
    if (tiles.size() >= (size_t)INT32_MAX) return fail(AZI_EOVERFLOW, "too many tiles");
    AZI_HIP(b->tiles.upload(tiles.data(), tiles.size() * sizeof(azi::Tile), b->device), "tiles");
    AZI_HIP(b->splits.upload(splits.data(), splits.size() * sizeof(azi::Split), b->device),
            "splits");
    AZI_HIP(b->parts.alloc((size_t)std::max(nparts, 1) * 16, b->device), "partials");
    b->ntiles = (int32_t)tiles.size();
    b->nsplits = (int32_t)splits.size();
    b->nparts = nparts;
    return AZI_OK;
}

// Instance-relative row pointers of a batch, rebuilt from the global ones.
void batch_local_indptr(const azi_batch* b, std::vector<std::vector<int32_t>>& store,
                        std::vector<const int32_t*>& ptrs, std::vector<int32_t>& npts) {
    store.resize(b->n);
    ptrs.resize(b->n);
    npts.resize(b->n);
    for (int32_t k = 0; k < b->n; ++k) {
        const int32_t nb = (int32_t)(b->bin_off[k + 1] - b->bin_off[k]);
        store[k].resize(nb + 1);
        for (int32_t r = 0; r <= nb; ++r)
            store[k][r] = b->rp_host[b->ip_off[k] + r] - (int32_t)b->nz_off[k];
        ptrs[k] = store[k].data();
        npts[k] = nb;
    }
}

int check_plan_ready(const azi_plan* p) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (p->device < 0) return fail(AZI_ESTATE, "plan is not on a device (azi_plan_upload)");
    return AZI_OK;
}

int upload_blocks(const azi::BlockMatrix& bm, int32_t dtype, int device, DevBuf& tiles,
                  DevBuf& rows, DevBuf& lp, DevBuf& coef, DevBuf& bin_ptr, DevBuf& parts) {
    if (bm.lp.size() >= (size_t)INT32_MAX || bm.rows.size() >= (size_t)INT32_MAX ||
        bm.tiles.size() >= (size_t)INT32_MAX)
        return fail(AZI_EOVERFLOW, "blocked matrix exceeds 2^31 entries, rows or tiles");
    AZI_HIP(tiles.upload(bm.tiles.data(), bm.tiles.size() * sizeof(azi::BlockTile), device),
            "block tiles");
    AZI_HIP(rows.upload(bm.rows.data(), bm.rows.size() * sizeof(azi::BlockRow), device),
            "block rows");
    AZI_HIP(lp.upload(bm.lp.data(), bm.lp.size() * 2, device), "block pixel ids");
    std::vector<char> c = to_storage(bm.coef.data(), (int64_t)bm.coef.size(),
                                     (int64_t)bm.coef.size(), dtype);
    AZI_HIP(coef.upload(c.data(), c.size(), device), "block coefficients");
    AZI_HIP(bin_ptr.upload(bm.bin_ptr.data(), bm.bin_ptr.size() * 4, device), "bin slots");
    AZI_HIP(parts.alloc(std::max<size_t>(bm.rows.size(), 1) * 16, device), "block partials");
    return AZI_OK;
}

// The band layout in either encoding (per entry, or per run).
bool is_band(int32_t layout) { return layout == AZI_LAYOUT_BAND || layout == AZI_LAYOUT_RUN; }

// Run layout: neighbouring bands co-scheduled per workgroup (tiling band
// 16 or 32 = 4 or 8 bands of 4 bins), else one band per workgroup.
int32_t run_waves(const azi_tiling& t) { return t.band == 16 ? 4 : t.band == 32 ? 8 : 1; }

int32_t band_rows_of(const azi_tiling& t) {
    return (t.band == 4 || t.band == 8 || t.band == 16) ? t.band : 8;
}

int32_t max_count_of(const std::vector<int32_t>& bin_count) {
    int32_t m = 0;
    for (int32_t c : bin_count) m = std::max(m, c);
    return m;
}

int upload_bands(const azi::BandMatrix& bm, int32_t dtype, int device, DevBuf& pieces,
                 DevBuf& packed, DevBuf& coef, DevBuf& bin_slot, DevBuf& bin_count,
                 DevBuf& parts, int32_t& max_count) {
    max_count = INT32_MAX;
    if (bm.packed.size() + kPad >= (size_t)INT32_MAX || bm.pieces.size() >= (size_t)INT32_MAX)
        return fail(AZI_EOVERFLOW, "band matrix exceeds 2^31 entries or pieces");
    AZI_HIP(pieces.upload(bm.pieces.data(), bm.pieces.size() * sizeof(azi::BandPiece), device),
            "band pieces");
    std::vector<int32_t> pk(bm.packed);
    pk.resize(pk.size() + kPad, 0);
    AZI_HIP(packed.upload(pk.data(), pk.size() * 4, device), "band entries");
    std::vector<char> c = to_storage(bm.coef.data(), (int64_t)bm.coef.size(),
                                     (int64_t)bm.coef.size() + kPad, dtype);
    AZI_HIP(coef.upload(c.data(), c.size(), device), "band coefficients");
    AZI_HIP(bin_slot.upload(bm.bin_slot.data(), bm.bin_slot.size() * 4, device), "bin slots");
    AZI_HIP(bin_count.upload(bm.bin_count.data(), bm.bin_count.size() * 4, device), "bin counts");
    AZI_HIP(parts.alloc((size_t)std::max(bm.nslots, 1) * 16, device), "band partials");
    max_count = max_count_of(bm.bin_count);
    return AZI_OK;
}

int plan_upload_bands(azi_plan* p) {
    p->rgbase.release();
    if (p->layout == AZI_LAYOUT_RUN) {
        try {
            azi::RunMatrix rm;
            if (!azi::build_runs(p->m, std::max(64, piece_nnz(p->tiling, p->m.nnz()) / 2), 0, 0, rm,
                                 nullptr,
                                 run_waves(p->tiling),
                                 balanced_tiles(p->tiling, p->device, run_waves(p->tiling),
                                                p->dtype, p->accum)))
                return fail(AZI_EOVERFLOW,
                            "the run layout takes images below 2^27 pixels and 2^31 entries");
            azi::BandMatrix bm;
            bm.pieces.swap(rm.pieces);
            bm.packed.swap(rm.runs);
            bm.coef.swap(rm.coef);
            bm.bin_slot.swap(rm.bin_slot);
            bm.bin_count.swap(rm.bin_count);
            bm.nslots = rm.nslots;
            p->band_rows = azi::kRunRows;
            int rc = upload_bands(bm, p->dtype, p->device, p->npieces_buf, p->npacked, p->ncoef,
                                  p->bin_slot, p->bin_count, p->nparts_buf, p->max_count);
            if (rc != AZI_OK) return rc;
            AZI_HIP(p->rgbase.upload(rm.gbase.data(), rm.gbase.size() * 4, p->device),
                    "run groups");
            p->npieces = (int32_t)bm.pieces.size();
        } catch (const std::bad_alloc&) {
            return fail(AZI_ENOMEM, "out of host memory building the run matrix");
        }
        return AZI_OK;
    }
    try {
        azi::BandMatrix bm;
        p->band_rows = band_rows_of(p->tiling);
        if (!azi::build_bands(p->m, p->band_rows, piece_nnz(p->tiling, p->m.nnz()), 0, 0, bm))
            return fail(AZI_EOVERFLOW, "the band layout takes images below 2^27 pixels");
        int rc = upload_bands(bm, p->dtype, p->device, p->npieces_buf, p->npacked, p->ncoef,
                              p->bin_slot, p->bin_count, p->nparts_buf, p->max_count);
        if (rc != AZI_OK) return rc;
        p->npieces = (int32_t)bm.pieces.size();
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the band matrix");
    }
    return AZI_OK;
}

azi::BandLaunch plan_band_args(const azi_plan* p, const void* x, void* I, void* W, void* U,
                               double empty) {
    azi::BandLaunch a;
    a.pieces = p->npieces_buf.as<azi::BandPiece>();
    a.npieces = p->npieces;
    a.packed = p->npacked.as<int32_t>();
    a.gbase = p->layout == AZI_LAYOUT_RUN ? p->rgbase.as<int32_t>() : nullptr;
    a.waves = p->layout == AZI_LAYOUT_RUN ? run_waves(p->tiling) : 1;
    a.coef = p->ncoef.p;
    a.bin_slot = p->bin_slot.as<int32_t>();
    a.bin_count = p->bin_count.as<int32_t>();
    a.max_count = p->max_count;
    a.R = p->band_rows;
    a.b0 = 0;
    a.b1 = p->m.npt;
    a.x = x;
    a.parts = p->nparts_buf.p;
    a.I = I;
    a.W = W;
    a.U = U;
    a.empty = empty;
    a.block = p->tiling.block;
    a.grid = p->tiling.grid;
    a.dtype = p->dtype;
    a.accum = p->accum;
    return a;
}

// Raw-frame band launch: cast and correction in the gather; with the
// normalisation folded (AZI_STAGE_FOLD) the folded coefficients, dark alone
// and the plan's U; with the dark term summed too (AZI_STAGE_FOLD_SUM,
// float64 sums) the raw count alone, the plan's D subtracted from W.
azi::BandLaunch plan_band_raw_args(const azi_plan* p, const void* raw, int32_t raw_dtype,
                                   void* I, void* W, void* U, double empty) {
    azi::BandLaunch a = plan_band_args(p, nullptr, I, W, U, empty);
    a.raw = raw;
    a.raw_dtype = raw_dtype;
    a.corr = (p->has_dark || p->has_norm) ? p->corr.p : nullptr;
    a.corr_kind = p->corr_kind;
    if (p->folded) {
        if (p->fcoef.p) a.coef = p->fcoef.p;
        a.ufix_in = p->ufix.as<double>();
        if (p->wdark.p) {  // the dark term is the plan's: the raw count alone
            a.corr = nullptr;
            a.wsub_in = p->wdark.as<double>();
        }
    }
    return a;
}

azi::BlockLaunch plan_block_args(const azi_plan* p, const void* img, int32_t img_dtype,
                                 bool correct, void* I, void* W, void* U, double empty) {
    azi::BlockLaunch a;
    a.tiles = p->btiles.as<azi::BlockTile>();
    a.ntiles = p->nbtiles;
    a.rows = p->brows.as<azi::BlockRow>();
    a.lp = p->blp.as<uint16_t>();
    a.coef = p->bcoef.p;
    a.bin_ptr = p->bin_ptr.as<int32_t>();
    a.b0 = 0;
    a.b1 = p->m.npt;
    a.img = img;
    a.img_dtype = img_dtype;
    if (correct && p->has_dark) a.dark = p->dark.p;
    if (correct && p->has_norm) a.norm = p->norm.p;
    a.parts = p->bparts.p;
    a.I = I;
    a.W = W;
    a.U = U;
    a.empty = empty;
    a.block = p->tiling.block;
    a.grid = p->tiling.grid;
    a.dtype = p->dtype;
    a.accum = p->accum;
    return a;
}

azi::FusedLaunch plan_fused_args(const azi_plan* p, const void* img, int32_t img_dtype,
                                 bool correct, void* I, void* W, void* U, double empty) {
    azi::FusedLaunch a;
    a.tiles = p->ftiles.as<azi::FusedTile>();
    a.ntiles = p->nftiles;
    a.slots = p->fslots.as<int32_t>();
    a.bin_ptr = p->fbin_ptr.as<int32_t>();
    a.geom = p->geom;
    a.unit = p->unit;
    a.split = p->split;
    a.pmin = p->m.pmin;
    a.delta = (p->m.pmax - p->m.pmin) / p->m.npt;
    a.npt = p->m.npt;
    a.img = img;
    a.img_dtype = img_dtype;
    if (correct && p->has_dark) a.dark = p->dark.p;
    if (correct && p->has_norm) a.norm = p->norm.p;
    a.parts = p->fparts.p;
    a.I = I;
    a.W = W;
    a.U = U;
    a.empty = empty;
    a.grid = p->tiling.grid;
    a.dtype = p->dtype;
    a.accum = p->accum;
    return a;
}

int plan_upload_fused(azi_plan* p) {
    try {
        std::vector<azi::FusedTile> tiles;
        std::vector<int32_t> slots, bin_ptr;
        azi::build_fused(p->m, p->geom.h, p->geom.w, tiles, slots, bin_ptr);
        if (tiles.size() >= (size_t)INT32_MAX || slots.size() >= (size_t)INT32_MAX)
            return fail(AZI_EOVERFLOW, "fused schedule exceeds 2^31 tiles or slots");
        AZI_HIP(p->ftiles.upload(tiles.data(), tiles.size() * sizeof(azi::FusedTile), p->device),
                "fused tiles");
        AZI_HIP(p->fslots.upload(slots.data(), slots.size() * 4, p->device), "fused slots");
        AZI_HIP(p->fbin_ptr.upload(bin_ptr.data(), bin_ptr.size() * 4, p->device), "fused bins");
        AZI_HIP(p->fparts.alloc(std::max<size_t>(slots.size(), 1) * 16, p->device),
                "fused partials");
        p->nftiles = (int32_t)tiles.size();
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the fused schedule");
    }
    return AZI_OK;
}

// (dark, 1 / norm) pairs for the band kernel's fused gather, formed when
// the plan integrates raw frames with AZI_STAGE_FUSE and has corrections;
// 12-byte records instead when the plan is float64 and its dark values are
// all floats.
// AZI_STAGE_FOLD on the run layout: every coefficient multiplied by its
// pixel's 1 / norm (on the host, from the plan's double coefficients,
// rounded once to the storage type), each run's dark value stored beside
// the run words, and the U of every bin summed once from the unfolded
// coefficients in the per-frame order (the kernels over any image, the
// reduction keeping U only).  AZI_STAGE_FOLD_SUM with float64 sums stores
// no dark value per run: D = (folded A) dark is summed once in the same
// order (the dark array as the image, the reduction keeping W only).
template <class S>
int download_as_double(const DevBuf& src, int64_t n, std::vector<double>& out, hipStream_t s) {
    std::vector<S> tmp((size_t)n);
    AZI_HIP(hipMemcpyAsync(tmp.data(), src.p, (size_t)n * sizeof(S), hipMemcpyDeviceToHost, s),
            "download corrections");
    AZI_HIP(hipStreamSynchronize(s), "download corrections");
    out.assign(tmp.begin(), tmp.end());
    return AZI_OK;
}

int plan_fold(azi_plan* p, hipStream_t s) {
    const int64_t npix = p->m.npix;
    const bool sum_dark = p->tiling.stage == AZI_STAGE_FOLD_SUM && p->accum == AZI_ACC_F64;
    try {
        std::vector<double> inv, dark;
        int rc = AZI_OK;
        if (p->has_norm) {
            rc = p->dtype == AZI_F64 ? download_as_double<double>(p->norm, npix, inv, s)
                                     : download_as_double<float>(p->norm, npix, inv, s);
            if (rc != AZI_OK) return rc;
            for (double& v : inv) v = 1.0 / v;
        }
        if (p->has_dark && !sum_dark) {
            rc = p->dtype == AZI_F64 ? download_as_double<double>(p->dark, npix, dark, s)
                                     : download_as_double<float>(p->dark, npix, dark, s);
            if (rc != AZI_OK) return rc;
        }
        azi::RunMatrix rm;
        if (!azi::build_runs(p->m, std::max(64, piece_nnz(p->tiling, p->m.nnz()) / 2), 0, 0, rm,
                             p->has_norm ? inv.data() : nullptr, run_waves(p->tiling)))
            return fail(AZI_EOVERFLOW,
                        "the run layout takes images below 2^27 pixels and 2^31 entries");
        if (p->has_norm) {
            std::vector<char> c = to_storage(rm.coef.data(), (int64_t)rm.coef.size(),
                                             (int64_t)rm.coef.size() + kPad, p->dtype);
            AZI_HIP(p->fcoef.upload(c.data(), c.size(), p->device), "folded coefficients");
        }
        if (p->has_dark && sum_dark) {
            p->corr_kind = azi::kCorrRunDark;  // no per-run array: D below
        } else if (p->has_dark) {
            // uint16 when every dark value is an integer count that fits
            // (its conversion to the storage type is exact: the same bits
            // from half the bytes), else float when every value is one
            // (always for float32 plans), else the storage type
            bool as_u16 = true, as_float = true;
            for (double d : dark) {
                as_u16 = as_u16 && d >= 0.0 && d <= 65535.0 && d == std::floor(d);
                as_float = as_float && (double)(float)d == d;
            }
            constexpr int32_t kPixMask = (1 << azi::kBandShift) - 1;
            const size_t nr = rm.runs.size() + kPad;
            if (as_u16) {
                std::vector<uint16_t> rd(nr, 0);
                for (size_t z = 0; z < rm.runs.size(); ++z)
                    if (rm.runs[z] >= 0)
                        rd[z] = (uint16_t)dark[(size_t)(rm.runs[z] & kPixMask)];
                AZI_HIP(p->corr.upload(rd.data(), rd.size() * 2, p->device), "run dark values");
                p->corr_kind = azi::kCorrRunDarkU16;
            } else {
                std::vector<double> rd(nr, 0.0);
                for (size_t z = 0; z < rm.runs.size(); ++z)
                    if (rm.runs[z] >= 0) rd[z] = dark[(size_t)(rm.runs[z] & kPixMask)];
                std::vector<char> c = to_storage(rd.data(), (int64_t)nr, (int64_t)nr,
                                                 as_float ? AZI_F32 : p->dtype);
                AZI_HIP(p->corr.upload(c.data(), c.size(), p->device), "run dark values");
                p->corr_kind = as_float && p->dtype == AZI_F64 ? azi::kCorrRunDarkF32
                                                               : azi::kCorrRunDark;
            }
        } else {
            p->corr_kind = azi::kCorrRunDark;
        }
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory folding the corrections");
    }
    AZI_HIP(p->ufix.alloc((size_t)p->m.npt * 8, p->device), "fixed U");
    azi::BandLaunch a = plan_band_args(p, p->xwork.p, nullptr, nullptr, nullptr, 0.0);
    a.ufix_out = p->ufix.as<double>();
    AZI_HIP(azi::launch_band(a, s), "fixed U");
    if (p->has_dark && sum_dark) {
        // D = (folded A) dark over the per-frame pieces, the dark array as
        // the image
        AZI_HIP(p->wdark.alloc((size_t)p->m.npt * 8, p->device), "fixed dark term");
        azi::BandLaunch d = plan_band_args(p, p->dark.p, nullptr, nullptr, nullptr, 0.0);
        if (p->fcoef.p) d.coef = p->fcoef.p;
        d.wfix_out = p->wdark.as<double>();
        AZI_HIP(azi::launch_band(d, s), "fixed dark term");
    }
    AZI_HIP(hipStreamSynchronize(s), "folded corrections");
    return AZI_OK;
}

int plan_corr_pair(azi_plan* p, hipStream_t s) {
    p->corr.release();
    p->fcoef.release();
    p->ufix.release();
    p->wdark.release();
    p->folded = false;
    p->corr_kind = azi::kCorrPair;
    if (!is_band(p->layout) || !gather_corrects(p->tiling.stage) ||
        !(p->has_dark || p->has_norm))
        return AZI_OK;
    if (p->layout == AZI_LAYOUT_RUN && folds(p->tiling.stage)) {
        const int rc = plan_fold(p, s);
        if (rc != AZI_OK) {
            p->corr.release();
            p->fcoef.release();
            p->ufix.release();
            p->wdark.release();
            p->corr_kind = azi::kCorrPair;
            return rc;
        }
        p->folded = true;
        return AZI_OK;
    }
    if (p->dtype == AZI_F64 && p->has_dark) {
        // float64 dark values that are all floats: 12-byte records
        DevBuf flag;
        int32_t h = 1;
        AZI_HIP(flag.alloc(4, p->device), "dark check");
        AZI_HIP(azi::launch_dark_is_float(p->dark.as<double>(), p->m.npix, flag.as<int32_t>(), s),
                "dark check");
        AZI_HIP(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s), "dark check");
        AZI_HIP(hipStreamSynchronize(s), "dark check");
        if (h == 0) {
            AZI_HIP(p->corr.alloc((size_t)p->m.npix * sizeof(azi::Corr12), p->device),
                    "correction records");
            AZI_HIP(azi::launch_corr_record12(p->dark.as<double>(),
                                              p->has_norm ? p->norm.as<double>() : nullptr,
                                              p->corr.p, p->m.npix, s), "correction records");
            AZI_HIP(hipStreamSynchronize(s), "correction records");
            p->corr_kind = azi::kCorrRecord12;
            return AZI_OK;
        }
    }
    AZI_HIP(p->corr.alloc((size_t)p->m.npix * 2 * elem_size(p->dtype), p->device),
            "correction pairs");
    AZI_HIP(azi::launch_corr_pair(p->has_dark ? p->dark.p : nullptr,
                                  p->has_norm ? p->norm.p : nullptr, p->corr.p, p->dtype,
                                  p->m.npix, s), "correction pairs");
    AZI_HIP(hipStreamSynchronize(s), "correction pairs");
    return AZI_OK;
}

// Staging of a (raw or corrected) row-major image into the plan's ring work
// image, with the plan's corrections when `correct` is set.
azi::StageLaunch plan_stage_args(const azi_plan* p, const void* img, int32_t img_dtype,
                                 bool correct) {
    azi::StageLaunch a;
    // AZI_STAGE_FUSE / _FOLD concern the band layouts; the ring staging then gathers
    a.mode = gather_corrects(p->tiling.stage) ? AZI_STAGE_GATHER : p->tiling.stage;
    a.raw = img;
    a.raw_dtype = img_dtype;
    a.order = p->order.as<int32_t>();
    a.pos = p->pos.as<int32_t>();
    a.tiles = p->stiles.as<azi::StageTile>();
    a.ntiles = p->nstiles;
    a.lidx = p->lidx.as<uint16_t>();
    a.dest = p->dest.as<int32_t>();
    const bool gather = a.mode == AZI_STAGE_GATHER;
    if (correct && p->has_dark) a.dark = gather ? p->dark_r.p : p->dark.p;
    if (correct && p->has_norm) a.norm = gather ? p->norm_r.p : p->norm.p;
    a.x = p->xwork.p;
    a.dtype = p->dtype;
    a.p0 = 0;
    a.p1 = gather ? p->used : p->m.npix;
    return a;
}

azi::ForwardLaunch plan_forward_args(const azi_plan* p, const void* x, void* I, void* W, void* U,
                                     double empty) {
    azi::ForwardLaunch a;
    a.tiles = p->tiles.as<azi::Tile>();
    a.ntiles = p->ntiles;
    a.splits = p->splits.as<azi::Split>();
    a.nsplits = p->nsplits;
    a.rowptr = p->rowptr.as<int32_t>();
    a.indices = p->indices.as<int32_t>();
    a.data = p->data.p;
    a.x = x;
    a.I = I;
    a.W = W;
    a.U = U;
    a.parts = p->parts.p;
    a.empty = empty;
    a.block = p->tiling.block;
    a.variant = p->tiling.variant;
    a.grid = p->tiling.grid;
    a.dtype = p->dtype;
    a.accum = p->accum;
    return a;
}

azi::ForwardLaunch batch_forward_args(const azi_batch* b, const void* x, void* I, void* W,
                                      void* U, double empty) {
    azi::ForwardLaunch a;
    a.tiles = b->tiles.as<azi::Tile>();
    a.ntiles = b->ntiles;
    a.splits = b->splits.as<azi::Split>();
    a.nsplits = b->nsplits;
    a.rowptr = b->rp.as<int32_t>();
    a.indices = b->indices.as<int32_t>();
    a.data = b->data.p;
    a.x = x;
    a.I = I;
    a.W = W;
    a.U = U;
    a.parts = b->parts.p;
    a.empty = empty;
    a.block = b->tiling.block;
    a.variant = b->tiling.variant;
    a.grid = b->tiling.grid;
    a.dtype = b->dtype;
    a.accum = b->accum;
    return a;
}

bool valid_raw_dtype(int32_t t) { return t >= AZI_I16 && t <= AZI_F64; }

}  // namespace

extern "C" {

int32_t azi_version(void) { return AZI_ABI_VERSION; }

const char* azi_last_error(void) { return g_err.c_str(); }

namespace {
int plan_build_device(azi_plan* p, int32_t npt, int32_t npt_azim, const double* range2,
                      int device, hipStream_t s);

// device < 0: the host builder; otherwise the device builder on that device,
// leaving the plan uploaded there.
int plan_create(const azi_geom* geom, int32_t npt, int32_t npt_azim, int32_t unit, int32_t split,
                const double* range2, int32_t dtype, int32_t accum, azi_plan** out,
                int32_t device = -1, hipStream_t stream = nullptr) {
    if (!geom || !out) return fail(AZI_EINVAL, "geom and out must not be NULL");
    *out = nullptr;
    if (geom->h < 1 || geom->w < 1) return fail(AZI_EINVAL, "image shape must be at least 1x1");
    if (npt < 1) return fail(AZI_EINVAL, "npt must be >= 1");
    if (npt_azim == 1 || npt_azim < 0) return fail(AZI_EINVAL, "npt_azim must be >= 2");
    if (!(geom->pixel_x_m > 0) || !(geom->pixel_y_m > 0) || !(geom->dist_m > 0) ||
        !(geom->wavelength_m > 0))
        return fail(AZI_EINVAL, "pixel sizes, distance and wavelength must be positive");
    if (!std::isfinite(geom->center_x_px) || !std::isfinite(geom->center_y_px))
        return fail(AZI_EINVAL, "beam centre must be finite");
    if (unit < AZI_UNIT_R_M || unit > AZI_UNIT_Q_NM) return fail(AZI_EINVAL, "unknown unit");
    if (split != AZI_SPLIT_NONE && split != AZI_SPLIT_BBOX && split != AZI_SPLIT_FULL)
        return fail(AZI_EINVAL, "unknown split");
    if (dtype != AZI_F32 && dtype != AZI_F64) return fail(AZI_EINVAL, "dtype must be AZI_F32 or AZI_F64");
    if (accum != AZI_ACC_F64 && accum != AZI_ACC_KAHAN32) return fail(AZI_EINVAL, "unknown accumulation");
    if (accum == AZI_ACC_KAHAN32 && dtype != AZI_F32)
        return fail(AZI_EINVAL, "Kahan float accumulation needs AZI_F32 storage");
    if (range2 && !(range2[1] > range2[0])) return fail(AZI_EINVAL, "range max must exceed min");
    std::unique_ptr<azi_plan> p(new (std::nothrow) azi_plan);
    if (!p) return fail(AZI_ENOMEM, "out of host memory");
    p->geom = *geom;
    p->dtype = dtype;
    p->accum = accum;
    if (dtype == AZI_F32) p->tiling = kDefaultTiling32;
    p->unit = unit;
    p->split = split;
    if (device >= 0) {
        const int rc = plan_build_device(p.get(), npt, npt_azim, range2, device, stream);
        if (rc != AZI_OK) return rc;
        *out = p.release();
        return AZI_OK;
    }
    std::string err;
    int rc;
    try {
        rc = azi::build_matrix(*geom, npt, npt_azim, unit, split, range2, p->m, err);
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the matrix");
    }
    if (rc != AZI_OK) return fail(rc, err);
    // the run layout numbers pixels in 27 bits; larger images take the CSR
    p->layout = p->m.npix < ((int64_t)1 << azi::kBandShift) ? AZI_LAYOUT_RUN : AZI_LAYOUT_PIXEL;
    if (p->m.two_d) {
        // short rows (tens of entries): the plain CSR with whole rows per
        // tile beats the band order, whose per-band pieces would be tiny
        p->layout = AZI_LAYOUT_PIXEL;
        p->tiling = kDefaultTiling2d;
    }
    *out = p.release();
    return AZI_OK;
}


int bit_length(int64_t v) {
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

extern "C++" {
template <class T>
int download(std::vector<T>& dst, const void* src, int64_t n, hipStream_t s) {
    dst.resize((size_t)n);
    if (n > 0)
        AZI_HIP(hipMemcpyAsync(dst.data(), src, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s),
                "download the matrix");
    return AZI_OK;
}
}  // extern "C++"

// Band layout from the pixel-major entries: a stable sort by band orders
// each band's entries by (pixel, bin); the pieces come from the band starts,
// which are the row pointers of the bands' first rows.
int plan_device_bands(azi_plan* p, const int32_t* rowidx, const int32_t* pix, const double* cdata,
                      int64_t nnz, DevBuf& work, DevBuf& skeys, DevBuf& perm, hipStream_t s) {
    const int32_t R = band_rows_of(p->tiling);
    p->band_rows = R;
    if (p->m.npix >= ((int64_t)1 << azi::kBandShift))
        return fail(AZI_EOVERFLOW, "the band layout takes images below 2^27 pixels");
    if (nnz + kPad >= (int64_t)INT32_MAX)
        return fail(AZI_EOVERFLOW, "band matrix exceeds 2^31 entries or pieces");
    const int32_t npt = p->m.npt;
    const int32_t nbands = (npt + R - 1) / R;
    const int dev = p->device;
    const size_t es = elem_size(p->dtype);
    DevBuf keys;
    AZI_HIP(keys.alloc((size_t)std::max<int64_t>(nnz, 1) * 4, dev), "band keys");
    AZI_HIP(azi::launch_div(rowidx, nnz, R, keys.as<int32_t>(), s), "band keys");
    AZI_HIP(azi::launch_sort(keys.as<int32_t>(), nnz, bit_length(nbands - 1), skeys.as<int32_t>(),
                             perm.as<int32_t>(), work.p, s), "band sort");
    AZI_HIP(p->npacked.alloc((size_t)(nnz + kPad) * 4, dev), "band entries");
    AZI_HIP(p->ncoef.alloc((size_t)(nnz + kPad) * es, dev), "band coefficients");
    AZI_HIP(azi::launch_band_entries(perm.as<int32_t>(), nnz, nnz + kPad, rowidx, pix, cdata, R,
                                     p->npacked.as<int32_t>(), p->ncoef.p, p->dtype, s),
            "band entries");
    try {
        std::vector<int64_t> start((size_t)nbands + 1);
        for (int32_t b = 0; b < nbands; ++b) start[b] = p->m.indptr[(size_t)b * R];
        start[nbands] = nnz;
        azi::BandMatrix bm;
        azi::band_pieces(start.data(), nbands, npt, R, piece_nnz(p->tiling, nnz), 0, 0, 0, bm);
        AZI_HIP(p->npieces_buf.upload(bm.pieces.data(), bm.pieces.size() * sizeof(azi::BandPiece),
                                      dev), "band pieces");
        AZI_HIP(p->bin_slot.upload(bm.bin_slot.data(), bm.bin_slot.size() * 4, dev), "bin slots");
        p->max_count = INT32_MAX;
        AZI_HIP(p->bin_count.upload(bm.bin_count.data(), bm.bin_count.size() * 4, dev),
                "bin counts");
        p->max_count = max_count_of(bm.bin_count);
        AZI_HIP(p->nparts_buf.alloc((size_t)std::max(bm.nslots, 1) * 16, dev), "band partials");
        p->npieces = (int32_t)bm.pieces.size();
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the band pieces");
    }
    AZI_HIP(hipStreamSynchronize(s), "band layout");
    return AZI_OK;
}

int plan_build_device(azi_plan* p, int32_t npt, int32_t npt_azim, const double* range2,
                      int device, hipStream_t s) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(AZI_EDEVICE, "no HIP device available");
    if (device >= count) return fail(AZI_EDEVICE, "no such HIP device");
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "set device");
    const azi_geom& g = p->geom;
    const int64_t npix = (int64_t)g.h * g.w;
    if (npix >= (int64_t)INT32_MAX) return fail(AZI_EOVERFLOW, "image has 2^31 pixels or more");
    const bool two_d = npt_azim > 0;
    if (two_d && (int64_t)npt * npt_azim >= (int64_t)INT32_MAX)
        return fail(AZI_EOVERFLOW, "npt_rad * npt_azim is 2^31 or more");
    p->device = device;
    azi::HostMatrix& m = p->m;
    m.npt_rad = npt;
    m.npt = two_d ? npt * npt_azim : npt;
    m.npt_azim = two_d ? npt_azim : 1;
    m.two_d = two_d;
    m.npix = npix;
    const bool boxes = p->split != AZI_SPLIT_NONE;
    const int64_t nblk = (npix + azi::kBuildBlock - 1) / azi::kBuildBlock;
    DevBuf lo, hi, bmin, bmax, r2, cnt, scanw, tot;
    AZI_HIP(lo.alloc((size_t)npix * 8, device), "extents");
    AZI_HIP(hi.alloc(boxes ? (size_t)npix * 8 : 8, device), "extents");
    AZI_HIP(bmin.alloc((size_t)nblk * 8, device), "block minima");
    AZI_HIP(bmax.alloc((size_t)nblk * 8, device), "block maxima");
    AZI_HIP(azi::launch_extents(g, p->unit, p->split, lo.as<double>(), hi.as<double>(),
                                bmin.as<double>(), bmax.as<double>(), s), "extents");
    double pr[2];
    if (range2) {
        pr[0] = range2[0];
        pr[1] = range2[1];
    } else {
        AZI_HIP(r2.alloc(16, device), "range");
        AZI_HIP(azi::launch_minmax(bmin.as<double>(), bmax.as<double>(), nblk, r2.as<double>(), s),
                "range");
        AZI_HIP(hipMemcpyAsync(pr, r2.p, 16, hipMemcpyDeviceToHost, s), "range");
        AZI_HIP(hipStreamSynchronize(s), "range");
    }
    if (!(pr[1] > pr[0]) || !std::isfinite(pr[0]) || !std::isfinite(pr[1]))
        return fail(AZI_EINVAL, "integration range is empty or not finite");
    m.pmin = pr[0];
    m.pmax = pr[1];
    const double delta = (m.pmax - m.pmin) / npt;
    AZI_HIP(cnt.alloc((size_t)npix * 4, device), "entry counts");
    const int32_t nazim = two_d ? npt_azim : 0;
    AZI_HIP(azi::launch_count(g, p->unit, p->split, lo.as<double>(), hi.as<double>(), m.pmin, delta,
                              npt, nazim, cnt.as<int32_t>(), s), "entry counts");
    AZI_HIP(p->colptr.alloc((size_t)(npix + 1) * 4, device), "colptr");
    AZI_HIP(scanw.alloc(azi::scan_work_bytes(npix), device), "scan work");
    AZI_HIP(tot.alloc(8, device), "scan total");
    AZI_HIP(azi::launch_scan(cnt.as<int32_t>(), npix, p->colptr.as<int32_t>(), tot.as<int64_t>(),
                             scanw.p, s), "scan");
    int64_t nnz = 0;
    AZI_HIP(hipMemcpyAsync(&nnz, tot.p, 8, hipMemcpyDeviceToHost, s), "scan total");
    AZI_HIP(hipStreamSynchronize(s), "scan total");
    if (nnz >= (int64_t)INT32_MAX - 2 * kPad)
        return fail(AZI_EOVERFLOW, "matrix has 2^31 nonzeros or more");
    cnt.release();
    const int64_t nnz_alloc = round_up(nnz, kPad) + kPad;
    const size_t es = elem_size(p->dtype);
    const size_t n1 = (size_t)std::max<int64_t>(nnz, 1);
    DevBuf cdata64, pix, work, skeys, perm, data64;
    AZI_HIP(p->rowidx.alloc(n1 * 4, device), "rowidx");
    AZI_HIP(cdata64.alloc(n1 * 8, device), "coefficients");
    AZI_HIP(pix.alloc(n1 * 4, device), "pixel ids");
    AZI_HIP(azi::launch_fill(g, p->unit, p->split, lo.as<double>(), hi.as<double>(), m.pmin, delta,
                             npt, nazim, p->colptr.as<int32_t>(), p->rowidx.as<int32_t>(),
                             cdata64.as<double>(), pix.as<int32_t>(), s), "fill");
    // bin-major order: stable sort of the pixel-major entries by bin
    AZI_HIP(work.alloc(azi::sort_work_bytes(nnz), device), "sort work");
    AZI_HIP(skeys.alloc(n1 * 4, device), "sorted bins");
    AZI_HIP(perm.alloc(n1 * 4, device), "permutation");
    AZI_HIP(azi::launch_sort(p->rowidx.as<int32_t>(), nnz, bit_length(m.npt - 1),
                             skeys.as<int32_t>(), perm.as<int32_t>(), work.p, s), "sort");
    AZI_HIP(p->rowptr.alloc((size_t)(m.npt + 1) * 4, device), "indptr");
    AZI_HIP(azi::launch_bounds(skeys.as<int32_t>(), nnz, m.npt, p->rowptr.as<int32_t>(), s),
            "indptr");
    AZI_HIP(p->indices.alloc((size_t)nnz_alloc * 4, device), "indices");
    AZI_HIP(p->data.alloc((size_t)nnz_alloc * es, device), "data");
    if (p->dtype != AZI_F64) AZI_HIP(data64.alloc(n1 * 8, device), "data (double)");
    AZI_HIP(azi::launch_gather(perm.as<int32_t>(), nnz, nnz_alloc, pix.as<int32_t>(),
                               cdata64.as<double>(), p->indices.as<int32_t>(), p->data.p,
                               p->dtype, p->dtype != AZI_F64 ? data64.as<double>() : nullptr, s),
            "gather");
    AZI_HIP(p->cdata.alloc((n1 + kAdjPad) * es, device), "cdata");
    AZI_HIP(azi::launch_to_storage(cdata64.as<double>(), nnz, p->cdata.p, p->dtype, s), "cdata");
    // host copy of the matrix, for export and for the host-side layouts
    try {
        int rc = download(m.colptr, p->colptr.p, npix + 1, s);
        if (rc == AZI_OK) rc = download(m.rowidx, p->rowidx.p, nnz, s);
        if (rc == AZI_OK) rc = download(m.cdata, cdata64.p, nnz, s);
        if (rc == AZI_OK) rc = download(m.indptr, p->rowptr.p, (int64_t)m.npt + 1, s);
        if (rc == AZI_OK) rc = download(m.indices, p->indices.p, nnz, s);
        if (rc == AZI_OK)
            rc = download(m.data, p->dtype == AZI_F64 ? p->data.p : data64.p, nnz, s);
        if (rc != AZI_OK) return rc;
        AZI_HIP(hipStreamSynchronize(s), "download the matrix");
        rc = upload_first(m, device, p->cfirst);
        if (rc != AZI_OK) return rc;
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory for the matrix copy");
    }
    data64.release();
    p->order.release();
    p->used = npix;
    AZI_HIP(p->xwork.alloc((size_t)npix * es, device), "work image");
    AZI_HIP(p->vwork.alloc((size_t)(m.npt + kAdjPad) * 8, device), "work vector");
    if (two_d) {
        // short rows: the plain CSR with whole rows per tile, as for
        // host-built two-dimensional plans
        p->layout = AZI_LAYOUT_PIXEL;
        p->tiling = kDefaultTiling2d;
        return plan_upload_tiles(p);
    }
    // the band layout's own bands of 4 bins (band 16 means four neighbouring
    // bands per workgroup only in the run layout)
    p->layout = AZI_LAYOUT_BAND;
    p->tiling.band = 4;
    int rc = plan_device_bands(p, p->rowidx.as<int32_t>(), pix.as<int32_t>(), cdata64.as<double>(),
                               nnz, work, skeys, perm, s);
    if (rc != AZI_OK) return rc;
    return plan_upload_tiles(p);
}
}  // namespace

int azi_plan_create(const azi_geom* geom, int32_t npt, int32_t unit, int32_t split,
                    const double* range2, int32_t dtype, int32_t accum, azi_plan** out) {
    return plan_create(geom, npt, 0, unit, split, range2, dtype, accum, out);
}

int azi_plan_create_device(const azi_geom* geom, int32_t npt, int32_t unit, int32_t split,
                           const double* range2, int32_t dtype, int32_t accum, int32_t device,
                           void* stream, azi_plan** out) {
    if (device < 0) {
        if (out) *out = nullptr;
        return fail(AZI_EDEVICE, "no such HIP device");
    }
    return plan_create(geom, npt, 0, unit, split, range2, dtype, accum, out, device,
                       static_cast<hipStream_t>(stream));
}

int azi_plan_create2d_device(const azi_geom* geom, int32_t npt_rad, int32_t npt_azim,
                             int32_t unit, int32_t split, const double* range2, int32_t dtype,
                             int32_t accum, int32_t device, void* stream, azi_plan** out) {
    if (device < 0) {
        if (out) *out = nullptr;
        return fail(AZI_EDEVICE, "no such HIP device");
    }
    if (npt_azim < 2) {
        if (out) *out = nullptr;
        return fail(AZI_EINVAL, "npt_azim must be >= 2");
    }
    return plan_create(geom, npt_rad, npt_azim, unit, split, range2, dtype, accum, out, device,
                       static_cast<hipStream_t>(stream));
}

int azi_plan_create2d(const azi_geom* geom, int32_t npt_rad, int32_t npt_azim, int32_t unit,
                      int32_t split, const double* range2, int32_t dtype, int32_t accum,
                      azi_plan** out) {
    if (npt_azim < 2) {
        if (out) *out = nullptr;
        return fail(AZI_EINVAL, "npt_azim must be >= 2");
    }
    return plan_create(geom, npt_rad, npt_azim, unit, split, range2, dtype, accum, out);
}

int azi_plan_destroy(azi_plan* plan) {
    delete plan;
    return AZI_OK;
}

int azi_plan_info(const azi_plan* p, int32_t* npt, int64_t* npix, int64_t* nnz, double* range2) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (npt) *npt = p->m.npt;
    if (npix) *npix = p->m.npix;
    if (nnz) *nnz = p->m.nnz();
    if (range2) {
        range2[0] = p->m.pmin;
        range2[1] = p->m.pmax;
    }
    return AZI_OK;
}

int azi_plan_positions(const azi_plan* p, double* pos) {
    if (!p || !pos) return fail(AZI_EINVAL, "plan and positions must not be NULL");
    const double delta = (p->m.pmax - p->m.pmin) / p->m.npt_rad;
    for (int32_t b = 0; b < p->m.npt_rad; ++b) pos[b] = p->m.pmin + (b + 0.5) * delta;
    return AZI_OK;
}

int azi_plan_shape(const azi_plan* p, int32_t* npt_rad, int32_t* npt_azim) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (npt_rad) *npt_rad = p->m.npt_rad;
    if (npt_azim) *npt_azim = p->m.two_d ? p->m.npt_azim : 0;
    return AZI_OK;
}

int azi_plan_azimuths(const azi_plan* p, double* chi) {
    if (!p || !chi) return fail(AZI_EINVAL, "plan and chi must not be NULL");
    if (!p->m.two_d) return fail(AZI_ESTATE, "the plan is one-dimensional");
    const double dchi = (2.0 * M_PI) / p->m.npt_azim;
    for (int32_t c = 0; c < p->m.npt_azim; ++c) chi[c] = -M_PI + (c + 0.5) * dchi;
    return AZI_OK;
}

int azi_plan_export_csr(const azi_plan* p, void* data, int32_t* indices, int32_t* indptr) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    const int64_t nnz = p->m.nnz();
    if (indptr) std::copy(p->m.indptr.begin(), p->m.indptr.end(), indptr);
    if (indices) std::copy(p->m.indices.begin(), p->m.indices.end(), indices);
    if (data) {
        if (p->dtype == AZI_F64) std::memcpy(data, p->m.data.data(), (size_t)nnz * 8);
        else for (int64_t k = 0; k < nnz; ++k) static_cast<float*>(data)[k] = (float)p->m.data[k];
    }
    return AZI_OK;
}

int azi_plan_export_csc(const azi_plan* p, void* data, int32_t* bins, int32_t* colptr) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    const int64_t nnz = p->m.nnz();
    if (colptr) std::copy(p->m.colptr.begin(), p->m.colptr.end(), colptr);
    if (bins) std::copy(p->m.rowidx.begin(), p->m.rowidx.end(), bins);
    if (data) {
        if (p->dtype == AZI_F64) std::memcpy(data, p->m.cdata.data(), (size_t)nnz * 8);
        else for (int64_t k = 0; k < nnz; ++k) static_cast<float*>(data)[k] = (float)p->m.cdata[k];
    }
    return AZI_OK;
}

int azi_plan_set_tiling(azi_plan* p, const azi_tiling* t) {
    if (!p || !t) return fail(AZI_EINVAL, "plan and tiling must not be NULL");
    if (!valid_tiling(*t)) return fail(AZI_EINVAL, kTilingRule);
    const bool retile = t->tile_nnz != p->tiling.tile_nnz || t->band != p->tiling.band;
    const bool restage = t->stage != p->tiling.stage;
    const bool reblock = t->block != p->tiling.block;
    p->tiling = *t;
    if (p->device >= 0 && retile) {
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(hipDeviceSynchronize(), "synchronise before retiling");
        if (is_band(p->layout)) {
            int rc = plan_upload_bands(p);
            if (rc != AZI_OK) return rc;
        }
        const int rc = plan_upload_tiles(p);
        if (rc != AZI_OK) return rc;
    }
    // the folded form's U follows the pieces and the workgroup size
    if (p->device >= 0 && (restage || (p->folded && (retile || reblock)))) {
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(hipDeviceSynchronize(), "synchronise before changing the stage");
        const int rc = plan_corr_pair(p, nullptr);
        if (rc != AZI_OK) return rc;
    }
    return AZI_OK;
}

int azi_plan_get_tiling(const azi_plan* p, azi_tiling* t, int32_t* ntiles) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (t) *t = p->tiling;
    if (ntiles) *ntiles = p->ntiles;
    return AZI_OK;
}

int azi_plan_tile_schedule(const azi_plan* p, const azi_tiling* tl, int32_t* ntiles,
                           int32_t* tiles, int32_t* nsplits, int32_t* splits) {
    if (!p || !tl) return fail(AZI_EINVAL, "plan and tiling must not be NULL");
    if (!valid_tiling(*tl)) return fail(AZI_EINVAL, kTilingRule);
    std::vector<azi::Tile> t;
    std::vector<azi::Split> sp;
    int32_t nparts = 0;
    azi::build_tiles(p->m.indptr.data(), p->m.npt, 0, 0, 0, piece_nnz(*tl, p->m.nnz()), tl->band,
                     t, sp, nparts);
    if (ntiles) *ntiles = (int32_t)t.size();
    if (nsplits) *nsplits = (int32_t)sp.size();
    if (tiles) std::memcpy(tiles, t.data(), t.size() * sizeof(azi::Tile));
    if (splits) std::memcpy(splits, sp.data(), sp.size() * sizeof(azi::Split));
    return AZI_OK;
}

int azi_plan_run_schedule(const azi_plan* p, int32_t tile_nnz, int64_t* nruns, int32_t* runs,
                          int32_t* gbase, double* coef, int32_t* npieces, int32_t* pieces,
                          int32_t* bin_slot, int32_t* bin_count) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (tile_nnz != 0 && (tile_nnz < 64 || tile_nnz > 16384))
        return fail(AZI_EINVAL, "tile_nnz must be 0 or in [64, 16384]");
    try {
        azi::RunMatrix rm;
        azi_tiling tl = p->tiling;
        tl.tile_nnz = tile_nnz;
        if (!azi::build_runs(p->m, std::max(64, piece_nnz(tl, p->m.nnz()) / 2), 0, 0, rm, nullptr,
                             run_waves(tl),
                             balanced_tiles(tl, p->device, run_waves(tl), p->dtype, p->accum)))
            return fail(AZI_EOVERFLOW,
                        "the run layout takes images below 2^27 pixels and 2^31 entries");
        if (nruns) *nruns = (int64_t)rm.runs.size();
        if (npieces) *npieces = (int32_t)rm.pieces.size();
        if (runs) std::copy(rm.runs.begin(), rm.runs.end(), runs);
        if (gbase) std::copy(rm.gbase.begin(), rm.gbase.end(), gbase);
        if (coef) std::copy(rm.coef.begin(), rm.coef.end(), coef);
        if (pieces)
            for (size_t k = 0; k < rm.pieces.size(); ++k) {
                const azi::BandPiece& pc = rm.pieces[k];
                const int32_t v[8] = {pc.z0, pc.z1, pc.bin0, pc.nrows, pc.slot0, 0, 0, 0};
                std::copy(v, v + 8, pieces + 8 * k);
            }
        if (bin_slot) std::copy(rm.bin_slot.begin(), rm.bin_slot.end(), bin_slot);
        if (bin_count) std::copy(rm.bin_count.begin(), rm.bin_count.end(), bin_count);
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the run matrix");
    }
    return AZI_OK;
}

int azi_plan_set_layout(azi_plan* p, int32_t layout) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (layout < AZI_LAYOUT_PIXEL || layout > AZI_LAYOUT_RUN)
        return fail(AZI_EINVAL, "layout must be one of AZI_LAYOUT_PIXEL/RING/TILE/BAND/FUSED/RUN");
    if (layout == AZI_LAYOUT_FUSED && (p->m.two_d || p->split == AZI_SPLIT_FULL))
        return fail(AZI_EINVAL,
                    "the fused layout takes one-dimensional plans without full splitting");
    if (layout == p->layout) return AZI_OK;
    // every check comes before the layout changes, so a refused call leaves
    // the plan as it was
    if (p->device >= 0 && (p->has_dark || p->has_norm))
        return fail(AZI_ESTATE, "set the layout before the corrections");
    const int32_t old = p->layout;
    p->layout = layout;
    if (p->device < 0) return AZI_OK;
    {
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) {
            p->layout = old;
            return hip_fail(g.err, "set device");
        }
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            p->layout = old;
            return hip_fail(e, "synchronise before re-upload");
        }
    }
    const int32_t dev = p->device;
    const int rc = azi_plan_upload(p, dev);
    if (rc == AZI_OK) return AZI_OK;
    // the new layout could not be placed: put the old one back
    const std::string why = azi_last_error();
    p->layout = old;
    const int rc2 = azi_plan_upload(p, dev);
    return fail(rc, why + (rc2 == AZI_OK
                               ? " (the plan keeps its previous layout)"
                               : " (the previous layout could not be restored either: the plan "
                                 "is no longer on a device)"));
}

int azi_plan_get_layout(const azi_plan* p, int32_t* layout) {
    if (!p || !layout) return fail(AZI_EINVAL, "plan and layout must not be NULL");
    *layout = p->layout;
    return AZI_OK;
}

int azi_plan_upload(azi_plan* p, int32_t device) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(AZI_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(AZI_EDEVICE, "no such HIP device");
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    p->device = device;
    auto body = [&]() -> int {
        const int64_t nnz = p->m.nnz();
        const int64_t nnz_alloc = round_up(nnz, kPad) + kPad;
        const size_t es = elem_size(p->dtype);
        try {
            std::vector<int32_t> idx((size_t)nnz_alloc, 0);
            const double* coef = p->m.data.data();
            azi::RingLayout ring;
            if (p->layout == AZI_LAYOUT_RING) {
                azi::build_ring(p->m, ring);
                std::copy(ring.indices.begin(), ring.indices.end(), idx.begin());
                coef = ring.data.data();
                AZI_HIP(p->order.upload(ring.order.data(), ring.order.size() * 4, device), "order");
                AZI_HIP(p->pos.upload(ring.pos.data(), ring.pos.size() * 4, device), "pos");
                std::vector<azi::StageTile> st;
                std::vector<uint16_t> lidx;
                std::vector<int32_t> dest;
                azi::build_stage_tiles(p->geom.h, p->geom.w, ring.pos.data(), 0, 0, 0, st, lidx,
                                       dest);
                AZI_HIP(p->stiles.upload(st.data(), st.size() * sizeof(azi::StageTile), device),
                        "stage tiles");
                AZI_HIP(p->lidx.upload(lidx.data(), lidx.size() * 2, device), "stage ranks");
                AZI_HIP(p->dest.upload(dest.data(), dest.size() * 4, device), "stage targets");
                p->nstiles = (int32_t)st.size();
                p->used = ring.used;
            } else {
                std::copy(p->m.indices.begin(), p->m.indices.end(), idx.begin());
                p->order.release();
                p->used = p->m.npix;
            }
            AZI_HIP(p->indices.upload(idx.data(), idx.size() * 4, device), "indices");
            std::vector<char> d = to_storage(coef, nnz, nnz_alloc, p->dtype);
            AZI_HIP(p->data.upload(d.data(), d.size(), device), "data");
            AZI_HIP(p->rowptr.upload(p->m.indptr.data(), p->m.indptr.size() * 4, device), "indptr");
            AZI_HIP(p->colptr.upload(p->m.colptr.data(), p->m.colptr.size() * 4, device), "colptr");
            AZI_HIP(p->rowidx.upload(p->m.rowidx.data(), (size_t)nnz * 4, device), "rowidx");
            const int rcf = upload_first(p->m, device, p->cfirst);
            if (rcf != AZI_OK) return rcf;
            std::vector<char> cd = to_storage(p->m.cdata.data(), nnz, nnz + kAdjPad, p->dtype);
            AZI_HIP(p->cdata.upload(cd.data(), cd.size(), device), "cdata");
        } catch (const std::bad_alloc&) {
            return fail(AZI_ENOMEM, "out of host memory staging the upload");
        }
        AZI_HIP(p->xwork.alloc((size_t)p->m.npix * es, device), "work image");
        AZI_HIP(p->vwork.alloc((size_t)(p->m.npt + kAdjPad) * 8, device), "work vector");
        if (is_band(p->layout)) {
            int rc2 = plan_upload_bands(p);
            if (rc2 != AZI_OK) return rc2;
        }
        if (p->layout == AZI_LAYOUT_FUSED) {
            int rc2 = plan_upload_fused(p);
            if (rc2 != AZI_OK) return rc2;
        }
        if (p->layout == AZI_LAYOUT_TILE) {
            try {
                azi::BlockMatrix bm;
                azi::build_blocks(p->m, p->geom.h, p->geom.w, 0, 0, bm);
                azi::finish_blocks(p->m.npt, bm);
                int rc2 = upload_blocks(bm, p->dtype, device, p->btiles, p->brows, p->blp,
                                        p->bcoef, p->bin_ptr, p->bparts);
                if (rc2 != AZI_OK) return rc2;
                p->nbtiles = (int32_t)bm.tiles.size();
            } catch (const std::bad_alloc&) {
                return fail(AZI_ENOMEM, "out of host memory building the blocked matrix");
            }
        }
        return plan_upload_tiles(p);
    };
    const int rc = body();
    if (rc != AZI_OK) p->device = -1;
    return rc;
}

int32_t azi_plan_correction_bytes(const azi_plan* p) {
    if (!p || !p->corr.p) return 0;
    if (p->corr_kind == azi::kCorrRecord12) return (int32_t)sizeof(azi::Corr12);
    if (p->corr_kind == azi::kCorrRunDarkU16) return 2;
    if (p->corr_kind == azi::kCorrRunDarkF32) return 4;
    if (p->corr_kind == azi::kCorrRunDark) return (int32_t)elem_size(p->dtype);
    return (int32_t)(2 * elem_size(p->dtype));
}

int64_t azi_plan_device_bytes(const azi_plan* p) {
    if (!p) return 0;
    const DevBuf* bufs[] = {&p->ftiles, &p->fslots, &p->fbin_ptr, &p->fparts, &p->corr, &p->cfirst,
                            &p->fcoef, &p->ufix, &p->wdark,
                            &p->rowptr, &p->indices, &p->data, &p->colptr, &p->rowidx,
                            &p->cdata, &p->tiles, &p->splits, &p->parts, &p->dark,
                            &p->norm, &p->xwork, &p->vwork, &p->order, &p->dark_r,
                            &p->norm_r, &p->pos, &p->stiles, &p->lidx, &p->dest,
                            &p->btiles, &p->brows, &p->blp, &p->bcoef, &p->bin_ptr,
                            &p->bparts, &p->npieces_buf, &p->npacked, &p->ncoef, &p->bin_slot,
                            &p->bin_count, &p->nparts_buf};
    int64_t s = 0;
    for (const DevBuf* b : bufs) s += (int64_t)b->bytes;
    return s;
}

int azi_plan_set_corrections(azi_plan* p, const void* dark, const void* flat, const void* solid,
                             const void* polar, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)p->m.npix * elem_size(p->dtype);
    AZI_HIP(hipStreamSynchronize(s), "synchronise before changing corrections");
    p->has_dark = false;
    p->has_norm = false;
    if (dark) {
        AZI_HIP(p->dark.alloc(bytes, p->device), "dark");
        AZI_HIP(hipMemcpyAsync(p->dark.p, dark, bytes, hipMemcpyDeviceToDevice, s), "copy dark");
        p->has_dark = true;
    } else {
        p->dark.release();
    }
    if (flat || solid || polar) {
        AZI_HIP(p->norm.alloc(bytes, p->device), "norm");
        AZI_HIP(azi::launch_norm(flat, solid, polar, p->norm.p, p->dtype, p->m.npix, s), "norm kernel");
        p->has_norm = true;
    } else {
        p->norm.release();
    }
    // ring-ordered copies for the ring layout's correction pass
    p->dark_r.release();
    p->norm_r.release();
    if (p->layout == AZI_LAYOUT_RING) {
        const int32_t st = p->dtype;
        if (p->has_dark) {
            AZI_HIP(p->dark_r.alloc(bytes, p->device), "dark (ring order)");
            AZI_HIP(azi::launch_correct(p->dark.p, st, p->order.as<int32_t>(), nullptr, nullptr,
                                        p->dark_r.p, st, p->used, s), "permute dark");
        }
        if (p->has_norm) {
            AZI_HIP(p->norm_r.alloc(bytes, p->device), "norm (ring order)");
            AZI_HIP(azi::launch_correct(p->norm.p, st, p->order.as<int32_t>(), nullptr, nullptr,
                                        p->norm_r.p, st, p->used, s), "permute norm");
        }
    }
    AZI_HIP(hipStreamSynchronize(s), "corrections");
    return plan_corr_pair(p, s);
}

int azi_correct(const azi_plan* p, const void* raw, int32_t raw_dtype, void* x, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!raw || !x) return fail(AZI_EINVAL, "raw and x must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    AZI_HIP(azi::launch_correct(raw, raw_dtype, nullptr, p->has_dark ? p->dark.p : nullptr,
                                p->has_norm ? p->norm.p : nullptr, x, p->dtype, p->m.npix,
                                static_cast<hipStream_t>(stream)),
            "correction kernel");
    return AZI_OK;
}

int azi_integrate1d(const azi_plan* p, const void* x, void* I, void* W, void* U, double empty,
                    void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->layout == AZI_LAYOUT_FUSED) {
        AZI_HIP(azi::launch_fused(plan_fused_args(p, x, p->dtype, false, I, W, U, empty), s),
                "fused forward kernels");
        return AZI_OK;
    }
    if (p->layout == AZI_LAYOUT_TILE) {
        AZI_HIP(azi::launch_block(plan_block_args(p, x, p->dtype, false, I, W, U, empty), s),
                "blocked forward kernels");
        return AZI_OK;
    }
    if (is_band(p->layout)) {
        AZI_HIP(azi::launch_band(plan_band_args(p, x, I, W, U, empty), s), "band forward kernels");
        return AZI_OK;
    }
    const void* xin = x;
    if (p->layout == AZI_LAYOUT_RING) {
        AZI_HIP(azi::launch_stage(plan_stage_args(p, x, p->dtype, false), s), "permutation kernel");
        xin = p->xwork.p;
    }
    AZI_HIP(azi::launch_forward(plan_forward_args(p, xin, I, W, U, empty), s), "forward kernel");
    return AZI_OK;
}

int azi_plan_stage(const azi_plan* p, const void* raw, int32_t raw_dtype, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!raw) return fail(AZI_EINVAL, "raw must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->layout == AZI_LAYOUT_RING) {
        AZI_HIP(azi::launch_stage(plan_stage_args(p, raw, raw_dtype, true), s), "staging kernel");
    } else {
        AZI_HIP(azi::launch_correct(raw, raw_dtype, nullptr, p->has_dark ? p->dark.p : nullptr,
                                    p->has_norm ? p->norm.p : nullptr, p->xwork.p, p->dtype,
                                    p->m.npix, s),
                "correction kernel");
    }
    return AZI_OK;
}

int azi_integrate1d_staged(const azi_plan* p, void* I, void* W, void* U, double empty,
                           void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!I) return fail(AZI_EINVAL, "out_I must not be NULL");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    if (p->layout == AZI_LAYOUT_FUSED) {
        AZI_HIP(azi::launch_fused(plan_fused_args(p, p->xwork.p, p->dtype, false, I, W, U, empty),
                                  static_cast<hipStream_t>(stream)),
                "fused forward kernels");
        return AZI_OK;
    }
    if (p->layout == AZI_LAYOUT_TILE) {
        AZI_HIP(azi::launch_block(plan_block_args(p, p->xwork.p, p->dtype, false, I, W, U, empty),
                                  static_cast<hipStream_t>(stream)),
                "blocked forward kernels");
        return AZI_OK;
    }
    if (is_band(p->layout)) {
        AZI_HIP(azi::launch_band(plan_band_args(p, p->xwork.p, I, W, U, empty),
                                 static_cast<hipStream_t>(stream)),
                "band forward kernels");
        return AZI_OK;
    }
    AZI_HIP(azi::launch_forward(plan_forward_args(p, p->xwork.p, I, W, U, empty),
                                static_cast<hipStream_t>(stream)),
            "forward kernel");
    return AZI_OK;
}

int azi_integrate1d_raw(const azi_plan* p, const void* raw, int32_t raw_dtype, void* I, void* W,
                        void* U, double empty, void* stream) {
    if (!I) return fail(AZI_EINVAL, "out_I must not be NULL");
    if (p && p->layout == AZI_LAYOUT_FUSED && p->device >= 0) {
        // cast, correction and integration in one kernel
        if (!raw) return fail(AZI_EINVAL, "raw must not be NULL");
        if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(azi::launch_fused(plan_fused_args(p, raw, raw_dtype, true, I, W, U, empty),
                                  static_cast<hipStream_t>(stream)),
                "fused forward kernels");
        return AZI_OK;
    }
    if (p && p->layout == AZI_LAYOUT_TILE && p->device >= 0) {
        // cast and correction fused into the blocked kernel
        if (!raw) return fail(AZI_EINVAL, "raw must not be NULL");
        if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(azi::launch_block(plan_block_args(p, raw, raw_dtype, true, I, W, U, empty),
                                  static_cast<hipStream_t>(stream)),
                "blocked forward kernels");
        return AZI_OK;
    }
    if (p && is_band(p->layout) && gather_corrects(p->tiling.stage) && p->device >= 0) {
        // cast and correction in the band kernel's gather
        if (!raw) return fail(AZI_EINVAL, "raw must not be NULL");
        if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(azi::launch_band(plan_band_raw_args(p, raw, raw_dtype, I, W, U, empty),
                                 static_cast<hipStream_t>(stream)),
                "band forward kernels");
        return AZI_OK;
    }
    int rc = azi_plan_stage(p, raw, raw_dtype, stream);
    if (rc != AZI_OK) return rc;
    return azi_integrate1d_staged(p, I, W, U, empty, stream);
}

}  // extern "C"

namespace {

// Partial sums of azi_integrate1d_raw_noalloc.  Each device that loads the
// library holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device.
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current; looked up
// on the first call for each device and kept.
int scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxScratchDevices)
        return fail(AZI_EDEVICE, "device ordinal beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        AZI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static scratch address");
        if (!ptr) return fail(AZI_EDEVICE, "static scratch address is NULL");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return AZI_OK;
}

}  // namespace

extern "C" {

int64_t azi_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

int azi_integrate1d_raw_noalloc(const azi_plan* p, const void* raw, int32_t raw_dtype, void* I,
                                void* W, void* U, double empty, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!raw || !I) return fail(AZI_EINVAL, "raw and out_I must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    // the layouts whose raw-frame path needs partial sums and nothing else
    size_t need = 0;
    if (is_band(p->layout) && gather_corrects(p->tiling.stage)) need = p->nparts_buf.bytes;
    else if (p->layout == AZI_LAYOUT_TILE) need = p->bparts.bytes;
    else if (p->layout == AZI_LAYOUT_FUSED) need = p->fparts.bytes;
    else
        return fail(AZI_EINVAL,
                    "the allocation-free call takes the run and band layouts (stage "
                    "AZI_STAGE_FUSE, _FOLD or _FOLD_SUM), the tile layout and the fused layout");
    if (need > kScratchBytes)
        return fail(AZI_EINVAL, "plan needs " + std::to_string(need) +
                                    " bytes of partial sums, more than the " +
                                    std::to_string(kScratchBytes) + "-byte static scratch");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    void* parts = nullptr;
    rc = scratch_address(p->device, &parts);
    if (rc != AZI_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->layout == AZI_LAYOUT_FUSED) {
        azi::FusedLaunch a = plan_fused_args(p, raw, raw_dtype, true, I, W, U, empty);
        a.parts = parts;
        AZI_HIP(azi::launch_fused(a, s), "fused forward kernels");
    } else if (p->layout == AZI_LAYOUT_TILE) {
        azi::BlockLaunch a = plan_block_args(p, raw, raw_dtype, true, I, W, U, empty);
        a.parts = parts;
        AZI_HIP(azi::launch_block(a, s), "blocked forward kernels");
    } else {
        azi::BandLaunch a = plan_band_raw_args(p, raw, raw_dtype, I, W, U, empty);
        a.parts = parts;
        AZI_HIP(azi::launch_band(a, s), "band forward kernels");
    }
    return AZI_OK;
}

int azi_integrate1d_backward(const azi_plan* p, const void* U, const void* gI, const void* gW,
                             void* gx, int32_t wrt_raw, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!gx) return fail(AZI_EINVAL, "grad_x must not be NULL");
    if (gI && !U) return fail(AZI_EINVAL, "U is needed with grad_I");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    azi::BackwardLaunch a;
    a.colptr = p->colptr.as<int32_t>();
    a.rowidx = p->rowidx.as<int32_t>();
    a.first = p->cfirst.as<int32_t>();
    a.cdata = p->cdata.p;
    a.U = U;
    a.gI = gI;
    a.gW = gW;
    a.norm = (wrt_raw && p->has_norm) ? p->norm.p : nullptr;
    a.v = p->vwork.as<double>();
    a.gx = gx;
    a.npix = p->m.npix;
    a.npt = p->m.npt;
    a.dtype = p->dtype;
    AZI_HIP(azi::launch_backward(a, static_cast<hipStream_t>(stream)), "backward kernels");
    return AZI_OK;
}

int azi_batch_create(azi_plan* const* plans, int32_t n, int32_t device, azi_batch** out) {
    if (!plans || !out || n < 1) return fail(AZI_EINVAL, "need n >= 1 plans and an out pointer");
    *out = nullptr;
    for (int32_t k = 0; k < n; ++k) {
        if (!plans[k]) return fail(AZI_EINVAL, "plan is NULL");
        if (plans[k]->dtype != plans[0]->dtype || plans[k]->accum != plans[0]->accum ||
            plans[k]->layout != plans[0]->layout)
            return fail(AZI_EINVAL, "plans of a batch must share dtype, accumulation and layout");
    if (plans[0]->layout == AZI_LAYOUT_FUSED)
        return fail(AZI_EINVAL, "batches take the pixel, ring, tile, band or run layout");
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(AZI_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(AZI_EDEVICE, "no such HIP device");
    std::unique_ptr<azi_batch> b(new (std::nothrow) azi_batch);
    if (!b) return fail(AZI_ENOMEM, "out of host memory");
    b->n = n;
    b->dtype = plans[0]->dtype;
    b->accum = plans[0]->accum;
    b->device = device;
    b->tiling = plans[0]->tiling;
    b->layout = plans[0]->layout;
    b->pix_off.assign(n + 1, 0);
    b->bin_off.assign(n + 1, 0);
    b->nz_off.assign(n + 1, 0);
    b->ip_off.assign(n + 1, 0);
    std::vector<int64_t> cz_off(n + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        const azi::HostMatrix& m = plans[k]->m;
        b->pix_off[k + 1] = b->pix_off[k] + m.npix;
        b->bin_off[k + 1] = b->bin_off[k] + m.npt;
        b->nz_off[k + 1] = b->nz_off[k] + round_up(m.nnz(), kPad);
        b->ip_off[k + 1] = b->ip_off[k] + m.npt + 1;
        cz_off[k + 1] = cz_off[k] + m.nnz();
    }
    b->npix = b->pix_off[n];
    b->npt = b->bin_off[n];
    b->nnz = cz_off[n];
    b->nnz_alloc = b->nz_off[n] + kPad;
    const int64_t lim = INT32_MAX;
    if (b->npix >= lim || b->npt >= lim || b->nnz_alloc >= lim || b->ip_off[n] >= lim)
        return fail(AZI_EOVERFLOW, "batch exceeds 2^31 pixels, bins or nonzeros");
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    const size_t es = elem_size(b->dtype);
    try {
        std::vector<int32_t> idx((size_t)b->nnz_alloc, 0);
        std::vector<char> dat((size_t)b->nnz_alloc * es, 0);
        b->rp_host.assign((size_t)b->ip_off[n], 0);
        const bool ring = b->layout == AZI_LAYOUT_RING;
        std::vector<int32_t> order(ring ? (size_t)b->npix : 0), pos(ring ? (size_t)b->npix : 0);
        std::vector<azi::StageTile> st;
        std::vector<uint16_t> lidx;
        std::vector<int32_t> dest;
        b->stile_off.assign(n + 1, 0);
        for (int32_t k = 0; k < n; ++k) {
            const azi::HostMatrix& m = plans[k]->m;
            const int64_t z0 = b->nz_off[k];
            const int32_t po = (int32_t)b->pix_off[k];
            azi::RingLayout rl;
            if (ring) {
                azi::build_ring(m, rl);
                for (int64_t q = 0; q < m.npix; ++q) {
                    order[po + q] = rl.order[q] + po;
                    pos[po + q] = rl.pos[q] + po;
                }
                b->stile_off[k] = (int64_t)st.size();
                azi::build_stage_tiles(plans[k]->geom.h, plans[k]->geom.w, rl.pos.data(), po, po, 0,
                                       st, lidx, dest);
                b->stile_off[k + 1] = (int64_t)st.size();
            }
            const int32_t* cols = ring ? rl.indices.data() : m.indices.data();
            const double* coef = ring ? rl.data.data() : m.data.data();
            for (int64_t e = 0; e < m.nnz(); ++e) {
                idx[z0 + e] = cols[e] + po;
                if (b->dtype == AZI_F64) reinterpret_cast<double*>(dat.data())[z0 + e] = coef[e];
                else reinterpret_cast<float*>(dat.data())[z0 + e] = (float)coef[e];
            }
            for (int32_t r = 0; r <= m.npt; ++r)
                b->rp_host[b->ip_off[k] + r] = m.indptr[r] + (int32_t)z0;
        }
        b->cz_off = cz_off;
        if (is_band(b->layout)) {
            std::vector<const azi::HostMatrix*> ms(n);
            for (int32_t k = 0; k < n; ++k) ms[k] = &plans[k]->m;
            int rc2 = batch_build_bands(b.get(), ms);
            if (rc2 != AZI_OK) return rc2;
        }
        if (b->layout == AZI_LAYOUT_TILE) {
            azi::BlockMatrix bm;
            b->btile_off.assign(n + 1, 0);
            for (int32_t k = 0; k < n; ++k) {
                b->btile_off[k] = (int64_t)bm.tiles.size();
                azi::build_blocks(plans[k]->m, plans[k]->geom.h, plans[k]->geom.w, b->pix_off[k],
                                  b->bin_off[k], bm);
            }
            b->btile_off[n] = (int64_t)bm.tiles.size();
            azi::finish_blocks(b->npt, bm);
            int rc2 = upload_blocks(bm, b->dtype, device, b->btiles, b->brows, b->blp, b->bcoef,
                                    b->bin_ptr, b->bparts);
            if (rc2 != AZI_OK) return rc2;
            b->nbtiles = (int32_t)bm.tiles.size();
        }
        if (ring) {
            AZI_HIP(b->order.upload(order.data(), order.size() * 4, device), "order");
            AZI_HIP(b->pos.upload(pos.data(), pos.size() * 4, device), "pos");
            AZI_HIP(b->stiles.upload(st.data(), st.size() * sizeof(azi::StageTile), device),
                    "stage tiles");
            AZI_HIP(b->lidx.upload(lidx.data(), lidx.size() * 2, device), "stage ranks");
            AZI_HIP(b->dest.upload(dest.data(), dest.size() * 4, device), "stage targets");
        }
        AZI_HIP(b->xwork.alloc((size_t)b->npix * es, device), "work image");
        AZI_HIP(b->indices.upload(idx.data(), idx.size() * 4, device), "indices");
        AZI_HIP(b->data.upload(dat.data(), dat.size(), device), "data");
        AZI_HIP(b->rp.upload(b->rp_host.data(), b->rp_host.size() * 4, device), "row pointers");
        std::vector<int32_t>().swap(idx);
        std::vector<char>().swap(dat);
        std::vector<int32_t> colptr((size_t)b->npix + 1, 0), rowidx((size_t)b->nnz, 0);
        std::vector<char> cdat((size_t)(std::max<int64_t>(b->nnz, 1) + kAdjPad) * es, 0);
        for (int32_t k = 0; k < n; ++k) {
            const azi::HostMatrix& m = plans[k]->m;
            for (int64_t p = 0; p < m.npix; ++p)
                colptr[b->pix_off[k] + p] = m.colptr[p] + (int32_t)cz_off[k];
            for (int64_t e = 0; e < m.nnz(); ++e) {
                rowidx[cz_off[k] + e] = m.rowidx[e] + (int32_t)b->bin_off[k];
                if (b->dtype == AZI_F64) reinterpret_cast<double*>(cdat.data())[cz_off[k] + e] = m.cdata[e];
                else reinterpret_cast<float*>(cdat.data())[cz_off[k] + e] = (float)m.cdata[e];
            }
        }
        colptr[b->npix] = (int32_t)b->nnz;
        AZI_HIP(b->colptr.upload(colptr.data(), colptr.size() * 4, device), "colptr");
        AZI_HIP(b->rowidx.upload(rowidx.data(), rowidx.size() * 4, device), "rowidx");
        // first bins (global) when every instance has consecutive bins per pixel
        b->cfirst.release();
        std::vector<int32_t> first;
        for (int32_t k = 0; k < n; ++k) {
            const azi::HostMatrix& m = plans[k]->m;
            std::vector<int32_t> f = m.two_d ? std::vector<int32_t>() : consecutive_first(m);
            if (f.empty() && m.npix > 0) {
                first.clear();
                break;
            }
            for (int32_t& v : f) v += (int32_t)b->bin_off[k];
            first.insert(first.end(), f.begin(), f.end());
        }
        if ((int64_t)first.size() == b->npix)
            AZI_HIP(b->cfirst.upload(first.data(), first.size() * 4, device), "first bins");
        AZI_HIP(b->cdata.upload(cdat.data(), cdat.size(), device), "cdata");
        AZI_HIP(b->vwork.alloc((size_t)(b->npt + kAdjPad) * 8, device), "work vector");
        std::vector<std::vector<int32_t>> store;
        std::vector<const int32_t*> ptrs;
        std::vector<int32_t> npts;
        batch_local_indptr(b.get(), store, ptrs, npts);
        int rc = batch_upload_tiles(b.get(), ptrs, npts);
        if (rc != AZI_OK) return rc;
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory staging the batch");
    }
    *out = b.release();
    return AZI_OK;
}

int azi_batch_destroy(azi_batch* b) {
    delete b;
    return AZI_OK;
}

int azi_batch_info(const azi_batch* b, int32_t* n, int64_t* npix, int64_t* npt, int64_t* nnz,
                   int64_t* pix_off, int64_t* bin_off) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (n) *n = b->n;
    if (npix) *npix = b->npix;
    if (npt) *npt = b->npt;
    if (nnz) *nnz = b->nnz;
    if (pix_off) std::copy(b->pix_off.begin(), b->pix_off.end(), pix_off);
    if (bin_off) std::copy(b->bin_off.begin(), b->bin_off.end(), bin_off);
    return AZI_OK;
}

int azi_batch_set_tiling(azi_batch* b, const azi_tiling* t) {
    if (!b || !t) return fail(AZI_EINVAL, "batch and tiling must not be NULL");
    if (!valid_tiling(*t)) return fail(AZI_EINVAL, kTilingRule);
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    const bool retile =
        t->tile_nnz != b->tiling.tile_nnz || t->band != b->tiling.band || b->ntiles == 0;
    b->tiling = *t;
    if (retile) {
        AZI_HIP(hipDeviceSynchronize(), "synchronise before retiling");
        if (is_band(b->layout) && b->npieces_buf.p) {
            int rc = batch_rebuild_bands(b);
            if (rc != AZI_OK) return rc;
        }
        std::vector<std::vector<int32_t>> store;
        std::vector<const int32_t*> ptrs;
        std::vector<int32_t> npts;
        batch_local_indptr(b, store, ptrs, npts);
        return batch_upload_tiles(b, ptrs, npts);
    }
    return AZI_OK;
}

int azi_batch_get_tiling(const azi_batch* b, azi_tiling* t, int32_t* ntiles) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (t) *t = b->tiling;
    if (ntiles) *ntiles = b->ntiles;
    return AZI_OK;
}

}  // extern "C"

namespace {

// Brings a batch's images into its work image (ring positions, or a cast
// copy), instance range [k0, k1) only.
int batch_build_bands(azi_batch* b, const std::vector<const azi::HostMatrix*>& ms) {
    b->rgbase.release();
    if (b->layout == AZI_LAYOUT_RUN) {
        azi::RunMatrix rm;
        b->band_rows = azi::kRunRows;
        b->piece_off.assign(b->n + 1, 0);
        for (int32_t k = 0; k < b->n; ++k) {
            b->piece_off[k] = (int64_t)rm.pieces.size();
            if (!azi::build_runs(*ms[k], std::max(64, piece_nnz(b->tiling, ms[k]->nnz()) / 2),
                                 b->pix_off[k], b->bin_off[k], rm, nullptr,
                                 run_waves(b->tiling)))
                return fail(AZI_EOVERFLOW,
                            "the run layout takes images below 2^27 pixels and 2^31 runs and "
                            "entries per batch");
        }
        b->piece_off[b->n] = (int64_t)rm.pieces.size();
        azi::BandMatrix bm;
        bm.pieces.swap(rm.pieces);
        bm.packed.swap(rm.runs);
        bm.coef.swap(rm.coef);
        bm.bin_slot.swap(rm.bin_slot);
        bm.bin_count.swap(rm.bin_count);
        bm.nslots = rm.nslots;
        int rc = upload_bands(bm, b->dtype, b->device, b->npieces_buf, b->npacked, b->ncoef,
                              b->bin_slot, b->bin_count, b->nparts_buf, b->max_count);
        if (rc != AZI_OK) return rc;
        AZI_HIP(b->rgbase.upload(rm.gbase.data(), rm.gbase.size() * 4, b->device), "run groups");
        b->npieces = (int32_t)bm.pieces.size();
        return AZI_OK;
    }
    azi::BandMatrix bm;
    b->band_rows = band_rows_of(b->tiling);
    b->piece_off.assign(b->n + 1, 0);
    for (int32_t k = 0; k < b->n; ++k) {
        b->piece_off[k] = (int64_t)bm.pieces.size();
        if (!azi::build_bands(*ms[k], b->band_rows, piece_nnz(b->tiling, ms[k]->nnz()),
                              b->pix_off[k],
                              b->bin_off[k], bm))
            return fail(AZI_EOVERFLOW, "the band layout takes images below 2^27 pixels");
    }
    b->piece_off[b->n] = (int64_t)bm.pieces.size();
    int rc = upload_bands(bm, b->dtype, b->device, b->npieces_buf, b->npacked, b->ncoef,
                          b->bin_slot, b->bin_count, b->nparts_buf, b->max_count);
    if (rc != AZI_OK) return rc;
    b->npieces = (int32_t)bm.pieces.size();
    return AZI_OK;
}

// Rebuilds a batch's bands (new band rows or piece size) from its device CSC.
int batch_rebuild_bands(azi_batch* b) {
    const size_t es = elem_size(b->dtype);
    std::vector<int32_t> colptr((size_t)b->npix + 1), rowidx((size_t)b->nnz);
    std::vector<char> cd((size_t)b->nnz * es);
    AZI_HIP(hipMemcpy(colptr.data(), b->colptr.p, colptr.size() * 4, hipMemcpyDeviceToHost),
            "download colptr");
    if (b->nnz > 0) {
        AZI_HIP(hipMemcpy(rowidx.data(), b->rowidx.p, rowidx.size() * 4, hipMemcpyDeviceToHost),
                "download rowidx");
        AZI_HIP(hipMemcpy(cd.data(), b->cdata.p, cd.size(), hipMemcpyDeviceToHost),
                "download cdata");
    }
    std::vector<azi::HostMatrix> ms(b->n);
    std::vector<const azi::HostMatrix*> ptrs(b->n);
    for (int32_t k = 0; k < b->n; ++k) {
        azi::HostMatrix& m = ms[k];
        m.npix = b->pix_off[k + 1] - b->pix_off[k];
        m.npt = (int32_t)(b->bin_off[k + 1] - b->bin_off[k]);
        const int64_t c0 = b->cz_off[k], c1 = b->cz_off[k + 1];
        m.colptr.resize(m.npix + 1);
        for (int64_t p = 0; p <= m.npix; ++p)
            m.colptr[p] = colptr[b->pix_off[k] + p] - (int32_t)c0;
        m.rowidx.resize(c1 - c0);
        m.cdata.resize(c1 - c0);
        m.indices.resize(c1 - c0);  // nnz() counts these
        for (int64_t e = c0; e < c1; ++e) {
            m.rowidx[e - c0] = rowidx[e] - (int32_t)b->bin_off[k];
            m.cdata[e - c0] = b->dtype == AZI_F64 ? reinterpret_cast<const double*>(cd.data())[e]
                                                  : (double)reinterpret_cast<const float*>(cd.data())[e];
        }
        ptrs[k] = &m;
    }
    return batch_build_bands(b, ptrs);
}

azi::BandLaunch batch_band_args(const azi_batch* b, const void* x, int32_t k0, int32_t k1,
                                void* I, void* W, void* U, double empty) {
    azi::BandLaunch a;
    a.pieces = b->npieces_buf.as<azi::BandPiece>() + b->piece_off[k0];
    a.npieces = (int32_t)(b->piece_off[k1] - b->piece_off[k0]);
    a.packed = b->npacked.as<int32_t>();
    a.gbase = b->layout == AZI_LAYOUT_RUN ? b->rgbase.as<int32_t>() : nullptr;
    a.waves = b->layout == AZI_LAYOUT_RUN ? run_waves(b->tiling) : 1;
    a.coef = b->ncoef.p;
    a.bin_slot = b->bin_slot.as<int32_t>();
    a.bin_count = b->bin_count.as<int32_t>();
    a.max_count = b->max_count;
    a.R = b->band_rows;
    a.b0 = b->bin_off[k0];
    a.b1 = b->bin_off[k1];
    a.x = x;
    a.parts = b->nparts_buf.p;
    a.I = I;
    a.W = W;
    a.U = U;
    a.empty = empty;
    a.block = b->tiling.block;
    a.grid = (k0 == 0 && k1 == b->n) ? b->tiling.grid : 0;
    a.dtype = b->dtype;
    a.accum = b->accum;
    return a;
}

azi::BlockLaunch batch_block_args(const azi_batch* b, const void* img, int32_t img_dtype,
                                  int32_t k0, int32_t k1, void* I, void* W, void* U,
                                  double empty) {
    azi::BlockLaunch a;
    a.tiles = b->btiles.as<azi::BlockTile>() + b->btile_off[k0];
    a.ntiles = (int32_t)(b->btile_off[k1] - b->btile_off[k0]);
    a.rows = b->brows.as<azi::BlockRow>();
    a.lp = b->blp.as<uint16_t>();
    a.coef = b->bcoef.p;
    a.bin_ptr = b->bin_ptr.as<int32_t>();
    a.b0 = b->bin_off[k0];
    a.b1 = b->bin_off[k1];
    a.img = img;
    a.img_dtype = img_dtype;
    a.parts = b->bparts.p;
    a.I = I;
    a.W = W;
    a.U = U;
    a.empty = empty;
    a.block = b->tiling.block;
    a.grid = (k0 == 0 && k1 == b->n) ? b->tiling.grid : 0;
    a.dtype = b->dtype;
    a.accum = b->accum;
    return a;
}

int batch_stage(azi_batch* b, const void* img, int32_t img_dtype, int32_t k0, int32_t k1,
                hipStream_t s) {
    const size_t es = elem_size(b->dtype);
    const int64_t p0 = b->pix_off[k0], p1 = b->pix_off[k1];
    if (b->layout != AZI_LAYOUT_RING) {
        // plain cast into the work image, same positions
        AZI_HIP(azi::launch_correct(static_cast<const char*>(img) + (size_t)p0 * elem_size_any(img_dtype),
                                    img_dtype, nullptr, nullptr, nullptr,
                                    static_cast<char*>(b->xwork.p) + (size_t)p0 * es, b->dtype,
                                    p1 - p0, s),
                "batch cast kernel");
        return AZI_OK;
    }
    azi::StageLaunch a;
    a.mode = gather_corrects(b->tiling.stage) ? AZI_STAGE_GATHER : b->tiling.stage;
    a.raw = img;
    a.raw_dtype = img_dtype;
    a.dtype = b->dtype;
    if (a.mode == AZI_STAGE_GATHER) {
        // order holds global pixel ids, so the source stays at the base
        a.order = b->order.as<int32_t>() + p0;
        a.x = static_cast<char*>(b->xwork.p) + (size_t)p0 * es;
        a.p0 = 0;
        a.p1 = p1 - p0;
    } else {
        a.pos = b->pos.as<int32_t>();
        a.tiles = b->stiles.as<azi::StageTile>() + b->stile_off[k0];
        a.ntiles = (int32_t)(b->stile_off[k1] - b->stile_off[k0]);
        a.lidx = b->lidx.as<uint16_t>();
        a.dest = b->dest.as<int32_t>();
        a.x = b->xwork.p;
        a.p0 = p0;
        a.p1 = p1;
    }
    AZI_HIP(azi::launch_stage(a, s), "batch staging kernel");
    return AZI_OK;
}

}  // namespace

extern "C" {

int azi_batch_forward(azi_batch* b, const void* x, void* I, void* W, void* U, double empty,
                      void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->layout == AZI_LAYOUT_TILE) {
        AZI_HIP(azi::launch_block(batch_block_args(b, x, b->dtype, 0, b->n, I, W, U, empty), s),
                "batched blocked kernels");
        return AZI_OK;
    }
    if (is_band(b->layout)) {
        AZI_HIP(azi::launch_band(batch_band_args(b, x, 0, b->n, I, W, U, empty), s),
                "batched band kernels");
        return AZI_OK;
    }
    const void* xin = x;
    if (b->layout == AZI_LAYOUT_RING) {
        int rc = batch_stage(b, x, b->dtype, 0, b->n, s);
        if (rc != AZI_OK) return rc;
        xin = b->xwork.p;
    }
    AZI_HIP(azi::launch_forward(batch_forward_args(b, xin, I, W, U, empty), s),
            "batched forward kernel");
    return AZI_OK;
}

int azi_batch_forward_raw(azi_batch* b, const void* raw, int32_t raw_dtype, void* I, void* W,
                          void* U, double empty, void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!raw || !I) return fail(AZI_EINVAL, "raw and out_I must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->layout == AZI_LAYOUT_TILE) {
        AZI_HIP(azi::launch_block(batch_block_args(b, raw, raw_dtype, 0, b->n, I, W, U, empty), s),
                "batched blocked kernels");
        return AZI_OK;
    }
    if (is_band(b->layout) && gather_corrects(b->tiling.stage)) {
        azi::BandLaunch a = batch_band_args(b, nullptr, 0, b->n, I, W, U, empty);
        a.raw = raw;
        a.raw_dtype = raw_dtype;
        AZI_HIP(azi::launch_band(a, s), "batched band kernels");
        return AZI_OK;
    }
    int rc = batch_stage(b, raw, raw_dtype, 0, b->n, s);
    if (rc != AZI_OK) return rc;
    if (is_band(b->layout)) {
        AZI_HIP(azi::launch_band(batch_band_args(b, b->xwork.p, 0, b->n, I, W, U, empty), s),
                "batched band kernels");
        return AZI_OK;
    }
    AZI_HIP(azi::launch_forward(batch_forward_args(b, b->xwork.p, I, W, U, empty), s),
            "batched forward kernel");
    return AZI_OK;
}

int azi_batch_forward_loop(azi_batch* b, const void* x, void* I, void* W, void* U, double empty,
                           void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->layout == AZI_LAYOUT_TILE) {
        for (int32_t k = 0; k < b->n; ++k)
            AZI_HIP(azi::launch_block(batch_block_args(b, x, b->dtype, k, k + 1, I, W, U, empty), s),
                    "per-instance blocked kernels");
        return AZI_OK;
    }
    if (is_band(b->layout)) {
        for (int32_t k = 0; k < b->n; ++k)
            AZI_HIP(azi::launch_band(batch_band_args(b, x, k, k + 1, I, W, U, empty), s),
                    "per-instance band kernels");
        return AZI_OK;
    }
    azi::ForwardLaunch a = batch_forward_args(b, x, I, W, U, empty);
    a.grid = 0;
    if (b->layout == AZI_LAYOUT_RING) a.x = b->xwork.p;
    for (int32_t k = 0; k < b->n; ++k) {
        if (b->layout == AZI_LAYOUT_RING) {
            int rc = batch_stage(b, x, b->dtype, k, k + 1, s);
            if (rc != AZI_OK) return rc;
        }
        a.tiles = b->tiles.as<azi::Tile>() + b->tile_off[k];
        a.ntiles = (int32_t)(b->tile_off[k + 1] - b->tile_off[k]);
        a.splits = b->splits.as<azi::Split>() + b->split_off[k];
        a.nsplits = (int32_t)(b->split_off[k + 1] - b->split_off[k]);
        AZI_HIP(azi::launch_forward(a, s), "per-instance forward");
    }
    return AZI_OK;
}

int azi_batch_backward(azi_batch* b, const void* U, const void* gI, const void* gW, void* gx,
                       void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!gx) return fail(AZI_EINVAL, "grad_x must not be NULL");
    if (gI && !U) return fail(AZI_EINVAL, "U is needed with grad_I");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    azi::BackwardLaunch a;
    a.colptr = b->colptr.as<int32_t>();
    a.rowidx = b->rowidx.as<int32_t>();
    a.first = b->cfirst.as<int32_t>();
    a.cdata = b->cdata.p;
    a.U = U;
    a.gI = gI;
    a.gW = gW;
    a.norm = nullptr;
    a.v = b->vwork.as<double>();
    a.gx = gx;
    a.npix = b->npix;
    a.npt = b->npt;
    a.dtype = b->dtype;
    AZI_HIP(azi::launch_backward(a, static_cast<hipStream_t>(stream)), "batched backward");
    return AZI_OK;
}

int azi_batch_autotune(azi_batch* b, const void* x, void* I, void* W, void* U, void* stream,
                       char* report, int32_t report_len) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int ncu = 0;
    AZI_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device), "CU count");
    hipEvent_t e0, e1;
    AZI_HIP(hipEventCreate(&e0), "event");
    AZI_HIP(hipEventCreate(&e1), "event");
    // candidate tilings: the knobs that matter for the batch's layout
    std::vector<azi_tiling> cands;
    const int32_t st = b->tiling.stage;
    if (b->layout == AZI_LAYOUT_RUN) {
        // bands of 4 bins are fixed for runs; one band per workgroup of 128
        // or 256 threads, or four neighbouring bands per workgroup (band 16)
        for (int32_t tn : {1024, 2048, 4096, 8192, 16384}) {
            for (int32_t bl : {128, 256})
                for (int32_t gm : {0, 4, 8, 16})
                    cands.push_back(azi_tiling{tn, bl, 5, gm * ncu, 4, st});
            for (int32_t gm : {0, 8}) cands.push_back(azi_tiling{tn, 256, 5, gm * ncu, 16, st});
        }
    } else if (b->layout == AZI_LAYOUT_BAND) {
        for (int32_t tn : {1024, 2048, 4096, 8192})
            for (int32_t band : {4, 8})
                for (int32_t bl : {128, 256, 512})
                    for (int32_t gm : {0, 8}) cands.push_back(azi_tiling{tn, bl, 5, gm * ncu, band, st});
    } else if (b->layout == AZI_LAYOUT_TILE) {
        for (int32_t bl : {128, 256, 512})
            for (int32_t gm : {0, 4, 8})
                cands.push_back(azi_tiling{b->tiling.tile_nnz, bl, 5, gm * ncu, b->tiling.band, st});
    } else {
        for (int32_t tn : {512, 1024, 2048, 4096, 8192})
            for (int32_t band : {1, 4, 8, 16})
                for (int32_t bl : {128, 256, 512})
                    for (int32_t var : {2, 3, 5})
                        for (int32_t gm : {0, 8})
                            cands.push_back(azi_tiling{tn, bl, var, gm * ncu, band, st});
    }
    std::string rep = "{\"cus\": " + std::to_string(ncu) + ", \"candidates\": [";
    float best_ms = 1e30f;
    azi_tiling best_t = b->tiling;
    bool first = true;
    int rc = AZI_OK;
    for (const azi_tiling& cand : cands) {
        if (rc != AZI_OK) break;
        const int32_t tn = cand.tile_nnz, bl = cand.block, var = cand.variant, band = cand.band;

        rc = azi_batch_set_tiling(b, &cand);
        if (rc != AZI_OK) break;
        const int32_t units = is_band(b->layout)             ? b->npieces
                              : b->layout == AZI_LAYOUT_TILE ? b->nbtiles
                                                             : b->ntiles;
        if (cand.grid > 0 && cand.grid >= units) continue;  // same as one per unit
        hipError_t e = hipSuccess;
        // warm-up, then the best of 5 timed runs of the batch's own forward
        if (azi_batch_forward(b, x, I, W, U, 0.0, s) != AZI_OK) e = hipErrorLaunchFailure;
        float best = 1e30f;
        for (int rep_i = 0; rep_i < 5 && e == hipSuccess; ++rep_i) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess && azi_batch_forward(b, x, I, W, U, 0.0, s) != AZI_OK)
                e = hipErrorLaunchFailure;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune launch");
            break;
        }
        char buf[224];
        std::snprintf(buf, sizeof buf,
                      "%s{\"tile_nnz\": %d, \"block\": %d, \"variant\": %d, \"grid\": %d, "
                      "\"band\": %d, \"tiles\": %d, \"ms\": %.5f}",
                      first ? "" : ", ", tn, bl, var, cand.grid, band, units, best);
        rep += buf;
        first = false;
        if (best < best_ms) {
            best_ms = best;
            best_t = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != AZI_OK) return rc;
    rc = azi_batch_set_tiling(b, &best_t);
    if (rc != AZI_OK) return rc;
    char buf[224];
    std::snprintf(buf, sizeof buf,
                  "], \"best\": {\"tile_nnz\": %d, \"block\": %d, \"variant\": %d, "
                  "\"grid\": %d, \"band\": %d, \"ms\": %.5f}}",
                  best_t.tile_nnz, best_t.block, best_t.variant, best_t.grid, best_t.band,
                  best_ms);
    rep += buf;
    if (report && report_len > 0) {
        const size_t n = std::min((size_t)report_len - 1, rep.size());
        std::memcpy(report, rep.data(), n);
        report[n] = '\0';
    }
    return AZI_OK;
}

int azi_plan_autotune(azi_plan* p, const void* x, void* I, void* W, void* U, void* stream,
                      char* report, int32_t report_len) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    struct Cand {
        int32_t layout;
        azi_tiling t;
    };
    const int32_t st = p->tiling.stage;
    // layouts change only while the plan has no corrections (they are tied
    // to the layout's pixel order)
    const bool relayout = !(p->has_dark || p->has_norm);
    std::vector<Cand> cands;
    auto add = [&](int32_t layout, int32_t tn, int32_t bl, int32_t var, int32_t band) {
        if (relayout || layout == p->layout) cands.push_back(Cand{layout, {tn, bl, var, 0, band, st}});
    };
    if (p->m.two_d) {
        for (int32_t var : {1, 2, 3, 5})
            for (int32_t tn : {2048, 4096, 8192})
                for (int32_t bl : {128, 256}) add(AZI_LAYOUT_PIXEL, tn, bl, var, 1);
        add(AZI_LAYOUT_RUN, 4096, 128, 5, 4);
        add(AZI_LAYOUT_RUN, 0, 256, 5, 16);
    } else {
        const bool runs_ok = p->m.npix < ((int64_t)1 << azi::kBandShift);
        if (runs_ok) {
            for (int32_t tn : {2048, 4096, 8192})
                for (int32_t bl : {128, 256}) add(AZI_LAYOUT_RUN, tn, bl, 5, 4);
            for (int32_t tn : {0, 2048, 4096, 8192})
                for (int32_t band : {16, 32}) add(AZI_LAYOUT_RUN, tn, 256, 5, band);
            for (int32_t tn : {2048, 4096})
                for (int32_t band : {4, 8}) add(AZI_LAYOUT_BAND, tn, 256, 5, band);
        }
        for (int32_t var : {2, 3, 5}) add(AZI_LAYOUT_PIXEL, 4096, 256, var, 1);
    }
    if (cands.empty()) cands.push_back(Cand{p->layout, p->tiling});
    static const char* const kNames[] = {"pixel", "ring", "tile", "band", "fused", "run"};
    hipEvent_t e0, e1;
    AZI_HIP(hipEventCreate(&e0), "event");
    AZI_HIP(hipEventCreate(&e1), "event");
    std::string rep = "{\"candidates\": [";
    float best_ms = 1e30f;
    Cand best = cands.front();
    for (size_t k = 0; k < cands.size() && rc == AZI_OK; ++k) {
        const Cand& c = cands[k];
        rc = azi_plan_set_layout(p, c.layout);
        if (rc == AZI_OK) rc = azi_plan_set_tiling(p, &c.t);
        if (rc != AZI_OK) break;
        hipError_t e = hipSuccess;
        if (azi_integrate1d(p, x, I, W, U, 0.0, s) != AZI_OK) e = hipErrorLaunchFailure;
        float ms_best = 1e30f;
        for (int rep_i = 0; rep_i < 5 && e == hipSuccess; ++rep_i) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess && azi_integrate1d(p, x, I, W, U, 0.0, s) != AZI_OK)
                e = hipErrorLaunchFailure;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            ms_best = std::min(ms_best, ms);
        }
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune launch");
            break;
        }
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "%s{\"layout\": \"%s\", \"tile_nnz\": %d, \"block\": %d, "
                      "\"variant\": %d, \"band\": %d, \"ms\": %.5f}",
                      k ? ", " : "", kNames[c.layout], c.t.tile_nnz, c.t.block, c.t.variant,
                      c.t.band, ms_best);
        rep += buf;
        if (ms_best < best_ms) {
            best_ms = ms_best;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != AZI_OK) return rc;
    rc = azi_plan_set_layout(p, best.layout);
    if (rc == AZI_OK) rc = azi_plan_set_tiling(p, &best.t);
    if (rc != AZI_OK) return rc;
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "], \"best\": {\"layout\": \"%s\", \"tile_nnz\": %d, \"block\": %d, "
                  "\"variant\": %d, \"band\": %d, \"ms\": %.5f}}",
                  kNames[best.layout], best.t.tile_nnz, best.t.block, best.t.variant, best.t.band,
                  best_ms);
    rep += buf;
    if (report && report_len > 0) {
        const size_t n = std::min((size_t)report_len - 1, rep.size());
        std::memcpy(report, rep.data(), n);
        report[n] = '\0';
    }
    return AZI_OK;
}

}  // extern "C"

namespace {

template <class F>
int capture(int device, hipStream_t user, F&& body, azi_graph** out) {
    (void)user;
    hipStream_t cs;
    AZI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "begin capture");
    }
    int rc = body(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc != AZI_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "instantiate graph");
    }
    azi_graph* gr = new (std::nothrow) azi_graph;
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(AZI_ENOMEM, "out of host memory");
    }
    gr->graph = graph;
    gr->exec = exec;
    gr->device = device;
    *out = gr;
    return AZI_OK;
}

}  // namespace

extern "C" {

int azi_graph_create_batch(azi_batch* b, const void* x, void* I, void* W, void* U, double empty,
                           const void* gI, const void* gW, void* gx, void* stream,
                           azi_graph** out) {
    if (!b || !out) return fail(AZI_EINVAL, "batch and out must not be NULL");
    *out = nullptr;
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    const bool bwd = gI || gW;
    if (bwd && !gx) return fail(AZI_EINVAL, "grad_x is needed with a backward");
    if (gI && !U) return fail(AZI_EINVAL, "out_U is needed with grad_I");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    return capture(b->device, static_cast<hipStream_t>(stream), [&](hipStream_t cs) {
        int rc = azi_batch_forward(b, x, I, W, U, empty, cs);
        if (rc == AZI_OK && bwd) rc = azi_batch_backward(b, U, gI, gW, gx, cs);
        return rc;
    }, out);
}

int azi_graph_create_plan(const azi_plan* p, const void* raw, int32_t raw_dtype, void* I, void* W,
                          void* U, double empty, void* stream, azi_graph** out) {
    if (!out) return fail(AZI_EINVAL, "out must not be NULL");
    *out = nullptr;
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    return capture(p->device, static_cast<hipStream_t>(stream), [&](hipStream_t cs) {
        return azi_integrate1d_raw(p, raw, raw_dtype, I, W, U, empty, cs);
    }, out);
}

int azi_graph_launch(azi_graph* gr, void* stream) {
    if (!gr) return fail(AZI_EINVAL, "graph is NULL");
    DeviceGuard g(gr->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    AZI_HIP(hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream)), "graph launch");
    return AZI_OK;
}

int azi_graph_destroy(azi_graph* gr) {
    if (!gr) return AZI_OK;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return AZI_OK;
}

}  // extern "C"
