// C ABI of the azimuthal-integration library (declared in include/azint.h):
// plan, batch and graph objects, device placement, argument checking and the
// per-frame entry points, which only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

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

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

size_t elem_size(int32_t dtype) { return dtype == AZI_F64 ? 8 : 4; }

bool valid_tiling(int32_t tile_nnz, int32_t block) {
    return tile_nnz >= 64 && tile_nnz <= 16384 && tile_nnz % 64 == 0 &&
           (block == 64 || block == 128 || block == 256 || block == 512);
}

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

}  // namespace

struct azi_plan {
    azi::HostMatrix m;
    int32_t dtype = AZI_F64, accum = AZI_ACC_F64, unit = 0, split = AZI_SPLIT_BBOX;
    int32_t tile_nnz = 2048, block = 256;
    int device = -1;
    DevBuf rowptr, indices, data, colptr, rowidx, cdata, tiles, splits, parts, dark, norm, xwork,
        vwork;
    int32_t ntiles = 0, nsplits = 0, nparts = 0;
    bool has_dark = false, has_norm = false;
};

struct azi_batch {
    int32_t n = 0, dtype = AZI_F64, accum = AZI_ACC_F64;
    int device = -1;
    int64_t npix = 0, npt = 0, nnz = 0, nnz_alloc = 0;
    std::vector<int64_t> pix_off, bin_off, nz_off, ip_off, tile_off, split_off;
    std::vector<int32_t> rp_host;  // concatenated row pointers, global nnz positions
    int32_t tile_nnz = 2048, block = 256, grid = 0;
    int32_t ntiles = 0, nsplits = 0, nparts = 0;
    DevBuf rp, indices, data, colptr, rowidx, cdata, tiles, splits, parts, vwork;
};

struct azi_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = -1;
};

namespace {

// (Re)builds and uploads the tile schedule of a plan.
int plan_upload_tiles(azi_plan* p) {
    std::vector<azi::Tile> tiles;
    std::vector<azi::Split> splits;
    int32_t nparts = 0;
    azi::build_tiles(p->m.indptr.data(), p->m.npt, 0, 0, 0, p->tile_nnz, tiles, splits, nparts);
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
        azi::build_tiles(indptrs[k], npts[k], b->nz_off[k], b->bin_off[k], b->ip_off[k],
                         b->tile_nnz, tiles, splits, nparts);
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
    a.block = p->block;
    a.grid = 0;
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
    a.block = b->block;
    a.grid = b->grid;
    a.dtype = b->dtype;
    a.accum = b->accum;
    return a;
}

bool valid_raw_dtype(int32_t t) { return t >= AZI_I16 && t <= AZI_F64; }

}  // namespace

extern "C" {

int32_t azi_version(void) { return AZI_ABI_VERSION; }

const char* azi_last_error(void) { return g_err.c_str(); }

int azi_plan_create(const azi_geom* geom, int32_t npt, int32_t unit, int32_t split,
                    const double* range2, int32_t dtype, int32_t accum, azi_plan** out) {
    if (!geom || !out) return fail(AZI_EINVAL, "geom and out must not be NULL");
    *out = nullptr;
    if (geom->h < 1 || geom->w < 1) return fail(AZI_EINVAL, "image shape must be at least 1x1");
    if (npt < 1) return fail(AZI_EINVAL, "npt must be >= 1");
    if (!(geom->pixel_x_m > 0) || !(geom->pixel_y_m > 0) || !(geom->dist_m > 0) ||
        !(geom->wavelength_m > 0))
        return fail(AZI_EINVAL, "pixel sizes, distance and wavelength must be positive");
    if (!std::isfinite(geom->center_x_px) || !std::isfinite(geom->center_y_px))
        return fail(AZI_EINVAL, "beam centre must be finite");
    if (unit < AZI_UNIT_R_M || unit > AZI_UNIT_Q_NM) return fail(AZI_EINVAL, "unknown unit");
    if (split != AZI_SPLIT_NONE && split != AZI_SPLIT_BBOX) return fail(AZI_EINVAL, "unknown split");
    if (dtype != AZI_F32 && dtype != AZI_F64) return fail(AZI_EINVAL, "dtype must be AZI_F32 or AZI_F64");
    if (accum != AZI_ACC_F64 && accum != AZI_ACC_KAHAN32) return fail(AZI_EINVAL, "unknown accumulation");
    if (accum == AZI_ACC_KAHAN32 && dtype != AZI_F32)
        return fail(AZI_EINVAL, "Kahan float accumulation needs AZI_F32 storage");
    if (range2 && !(range2[1] > range2[0])) return fail(AZI_EINVAL, "range max must exceed min");
    std::unique_ptr<azi_plan> p(new (std::nothrow) azi_plan);
    if (!p) return fail(AZI_ENOMEM, "out of host memory");
    p->dtype = dtype;
    p->accum = accum;
    p->unit = unit;
    p->split = split;
    std::string err;
    int rc;
    try {
        rc = azi::build_matrix(*geom, npt, unit, split, range2, p->m, err);
    } catch (const std::bad_alloc&) {
        return fail(AZI_ENOMEM, "out of host memory building the matrix");
    }
    if (rc != AZI_OK) return fail(rc, err);
    *out = p.release();
    return AZI_OK;
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
    const double delta = (p->m.pmax - p->m.pmin) / p->m.npt;
    for (int32_t b = 0; b < p->m.npt; ++b) pos[b] = p->m.pmin + (b + 0.5) * delta;
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

int azi_plan_set_tiling(azi_plan* p, int32_t tile_nnz, int32_t block) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (!valid_tiling(tile_nnz, block))
        return fail(AZI_EINVAL, "tile_nnz must be a multiple of 64 in [64, 16384] and block one of 64/128/256/512");
    p->tile_nnz = tile_nnz;
    p->block = block;
    if (p->device >= 0) {
        DeviceGuard g(p->device);
        if (g.err != hipSuccess) return hip_fail(g.err, "set device");
        AZI_HIP(hipDeviceSynchronize(), "synchronise before retiling");
        return plan_upload_tiles(p);
    }
    return AZI_OK;
}

int azi_plan_tile_schedule(const azi_plan* p, int32_t tile_nnz, int32_t* ntiles, int32_t* tiles,
                           int32_t* nsplits, int32_t* splits) {
    if (!p) return fail(AZI_EINVAL, "plan is NULL");
    if (!valid_tiling(tile_nnz, 256)) return fail(AZI_EINVAL, "bad tile_nnz");
    std::vector<azi::Tile> t;
    std::vector<azi::Split> sp;
    int32_t nparts = 0;
    azi::build_tiles(p->m.indptr.data(), p->m.npt, 0, 0, 0, tile_nnz, t, sp, nparts);
    if (ntiles) *ntiles = (int32_t)t.size();
    if (nsplits) *nsplits = (int32_t)sp.size();
    if (tiles) std::memcpy(tiles, t.data(), t.size() * sizeof(azi::Tile));
    if (splits) std::memcpy(splits, sp.data(), sp.size() * sizeof(azi::Split));
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
            std::copy(p->m.indices.begin(), p->m.indices.end(), idx.begin());
            AZI_HIP(p->indices.upload(idx.data(), idx.size() * 4, device), "indices");
            std::vector<char> d = to_storage(p->m.data.data(), nnz, nnz_alloc, p->dtype);
            AZI_HIP(p->data.upload(d.data(), d.size(), device), "data");
            AZI_HIP(p->rowptr.upload(p->m.indptr.data(), p->m.indptr.size() * 4, device), "indptr");
            AZI_HIP(p->colptr.upload(p->m.colptr.data(), p->m.colptr.size() * 4, device), "colptr");
            AZI_HIP(p->rowidx.upload(p->m.rowidx.data(), (size_t)nnz * 4, device), "rowidx");
            std::vector<char> cd = to_storage(p->m.cdata.data(), nnz, nnz, p->dtype);
            AZI_HIP(p->cdata.upload(cd.data(), cd.size(), device), "cdata");
        } catch (const std::bad_alloc&) {
            return fail(AZI_ENOMEM, "out of host memory staging the upload");
        }
        AZI_HIP(p->xwork.alloc((size_t)p->m.npix * es, device), "work image");
        AZI_HIP(p->vwork.alloc((size_t)p->m.npt * 8, device), "work vector");
        return plan_upload_tiles(p);
    };
    const int rc = body();
    if (rc != AZI_OK) p->device = -1;
    return rc;
}

int64_t azi_plan_device_bytes(const azi_plan* p) {
    if (!p) return 0;
    const DevBuf* bufs[] = {&p->rowptr, &p->indices, &p->data, &p->colptr, &p->rowidx,
                            &p->cdata, &p->tiles, &p->splits, &p->parts, &p->dark,
                            &p->norm, &p->xwork, &p->vwork};
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
    AZI_HIP(hipStreamSynchronize(s), "corrections");
    return AZI_OK;
}

int azi_correct(const azi_plan* p, const void* raw, int32_t raw_dtype, void* x, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!raw || !x) return fail(AZI_EINVAL, "raw and x must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    AZI_HIP(azi::launch_correct(raw, raw_dtype, p->has_dark ? p->dark.p : nullptr,
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
    AZI_HIP(azi::launch_forward(plan_forward_args(p, x, I, W, U, empty),
                                static_cast<hipStream_t>(stream)),
            "forward kernel");
    return AZI_OK;
}

int azi_integrate1d_raw(const azi_plan* p, const void* raw, int32_t raw_dtype, void* I, void* W,
                        void* U, double empty, void* stream) {
    int rc = check_plan_ready(p);
    if (rc != AZI_OK) return rc;
    if (!raw || !I) return fail(AZI_EINVAL, "raw and out_I must not be NULL");
    if (!valid_raw_dtype(raw_dtype)) return fail(AZI_EINVAL, "unknown raw dtype");
    DeviceGuard g(p->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    AZI_HIP(azi::launch_correct(raw, raw_dtype, p->has_dark ? p->dark.p : nullptr,
                                p->has_norm ? p->norm.p : nullptr, p->xwork.p, p->dtype,
                                p->m.npix, s),
            "correction kernel");
    AZI_HIP(azi::launch_forward(plan_forward_args(p, p->xwork.p, I, W, U, empty), s),
            "forward kernel");
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
        if (plans[k]->dtype != plans[0]->dtype || plans[k]->accum != plans[0]->accum)
            return fail(AZI_EINVAL, "plans of a batch must share dtype and accumulation");
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
    b->tile_nnz = plans[0]->tile_nnz;
    b->block = plans[0]->block;
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
        for (int32_t k = 0; k < n; ++k) {
            const azi::HostMatrix& m = plans[k]->m;
            const int64_t z0 = b->nz_off[k];
            for (int64_t e = 0; e < m.nnz(); ++e) {
                idx[z0 + e] = m.indices[e] + (int32_t)b->pix_off[k];
                if (b->dtype == AZI_F64) reinterpret_cast<double*>(dat.data())[z0 + e] = m.data[e];
                else reinterpret_cast<float*>(dat.data())[z0 + e] = (float)m.data[e];
            }
            for (int32_t r = 0; r <= m.npt; ++r)
                b->rp_host[b->ip_off[k] + r] = m.indptr[r] + (int32_t)z0;
        }
        AZI_HIP(b->indices.upload(idx.data(), idx.size() * 4, device), "indices");
        AZI_HIP(b->data.upload(dat.data(), dat.size(), device), "data");
        AZI_HIP(b->rp.upload(b->rp_host.data(), b->rp_host.size() * 4, device), "row pointers");
        std::vector<int32_t>().swap(idx);
        std::vector<char>().swap(dat);
        std::vector<int32_t> colptr((size_t)b->npix + 1, 0), rowidx((size_t)b->nnz, 0);
        std::vector<char> cdat((size_t)std::max<int64_t>(b->nnz, 1) * es, 0);
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
        AZI_HIP(b->cdata.upload(cdat.data(), (size_t)b->nnz * es, device), "cdata");
        AZI_HIP(b->vwork.alloc((size_t)b->npt * 8, device), "work vector");
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

int azi_batch_set_tiling(azi_batch* b, int32_t tile_nnz, int32_t block, int32_t grid) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!valid_tiling(tile_nnz, block) || grid < 0)
        return fail(AZI_EINVAL, "tile_nnz must be a multiple of 64 in [64, 16384], block one of 64/128/256/512, grid >= 0");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    AZI_HIP(hipDeviceSynchronize(), "synchronise before retiling");
    b->grid = grid;
    b->block = block;
    if (tile_nnz != b->tile_nnz || b->ntiles == 0) {
        b->tile_nnz = tile_nnz;
        std::vector<std::vector<int32_t>> store;
        std::vector<const int32_t*> ptrs;
        std::vector<int32_t> npts;
        batch_local_indptr(b, store, ptrs, npts);
        return batch_upload_tiles(b, ptrs, npts);
    }
    return AZI_OK;
}

int azi_batch_get_tiling(const azi_batch* b, int32_t* tile_nnz, int32_t* block, int32_t* grid,
                         int32_t* ntiles) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (tile_nnz) *tile_nnz = b->tile_nnz;
    if (block) *block = b->block;
    if (grid) *grid = b->grid;
    if (ntiles) *ntiles = b->ntiles;
    return AZI_OK;
}

int azi_batch_forward(azi_batch* b, const void* x, void* I, void* W, void* U, double empty,
                      void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    AZI_HIP(azi::launch_forward(batch_forward_args(b, x, I, W, U, empty),
                                static_cast<hipStream_t>(stream)),
            "batched forward kernel");
    return AZI_OK;
}

int azi_batch_forward_loop(azi_batch* b, const void* x, void* I, void* W, void* U, double empty,
                           void* stream) {
    if (!b) return fail(AZI_EINVAL, "batch is NULL");
    if (!x || !I) return fail(AZI_EINVAL, "x and out_I must not be NULL");
    DeviceGuard g(b->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "set device");
    azi::ForwardLaunch a = batch_forward_args(b, x, I, W, U, empty);
    a.grid = 0;
    for (int32_t k = 0; k < b->n; ++k) {
        a.tiles = b->tiles.as<azi::Tile>() + b->tile_off[k];
        a.ntiles = (int32_t)(b->tile_off[k + 1] - b->tile_off[k]);
        a.splits = b->splits.as<azi::Split>() + b->split_off[k];
        a.nsplits = (int32_t)(b->split_off[k + 1] - b->split_off[k]);
        AZI_HIP(azi::launch_forward(a, static_cast<hipStream_t>(stream)), "per-instance forward");
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
    const int32_t tiles_c[] = {512, 1024, 2048, 4096, 8192};
    const int32_t blocks_c[] = {128, 256, 512};
    const int32_t grids_m[] = {0, 4, 8, 16};
    std::string rep = "{\"cus\": " + std::to_string(ncu) + ", \"candidates\": [";
    float best_ms = 1e30f;
    int32_t bt = b->tile_nnz, bb = b->block, bg = b->grid;
    bool first = true;
    int rc = AZI_OK;
    for (int32_t tn : tiles_c) {
        for (int32_t bl : blocks_c) {
            for (int32_t gm : grids_m) {
                const int32_t grid = gm == 0 ? 0 : gm * ncu;
                rc = azi_batch_set_tiling(b, tn, bl, grid);
                if (rc != AZI_OK) break;
                if (grid > 0 && grid >= b->ntiles) continue;  // no different from one per tile
                azi::ForwardLaunch a = batch_forward_args(b, x, I, W, U, 0.0);
                hipError_t e = azi::launch_forward(a, s);  // warm-up
                float best = 1e30f;
                for (int rep_i = 0; rep_i < 5 && e == hipSuccess; ++rep_i) {
                    e = hipEventRecord(e0, s);
                    if (e == hipSuccess) e = azi::launch_forward(a, s);
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
                char buf[160];
                std::snprintf(buf, sizeof buf,
                              "%s{\"tile_nnz\": %d, \"block\": %d, \"grid\": %d, \"tiles\": %d, \"ms\": %.5f}",
                              first ? "" : ", ", tn, bl, grid, b->ntiles, best);
                rep += buf;
                first = false;
                if (best < best_ms) {
                    best_ms = best;
                    bt = tn;
                    bb = bl;
                    bg = grid;
                }
            }
            if (rc != AZI_OK) break;
        }
        if (rc != AZI_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != AZI_OK) return rc;
    rc = azi_batch_set_tiling(b, bt, bb, bg);
    if (rc != AZI_OK) return rc;
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "], \"best\": {\"tile_nnz\": %d, \"block\": %d, \"grid\": %d, \"ms\": %.5f}}",
                  bt, bb, bg, best_ms);
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
