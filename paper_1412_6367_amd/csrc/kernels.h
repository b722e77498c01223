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
    int32_t grid = 0;                  // 0: one workgroup per tile
    int32_t dtype = AZI_F64;
    int32_t accum = AZI_ACC_F64;
};

hipError_t launch_forward(const ForwardLaunch& a, hipStream_t s);

struct BackwardLaunch {
    const int32_t* colptr = nullptr;   // npix + 1 (global nnz positions)
    const int32_t* rowidx = nullptr;   // global bin ids
    const void* cdata = nullptr;       // storage type
    const void* U = nullptr;           // forward U, storage type
    const void* gI = nullptr;          // may be null
    const void* gW = nullptr;          // may be null
    const void* norm = nullptr;        // divide the result by it when non-null
    double* v = nullptr;               // work buffer, npt doubles
    void* gx = nullptr;                // npix, storage type
    int64_t npix = 0;
    int64_t npt = 0;
    int32_t dtype = AZI_F64;
};

hipError_t launch_backward(const BackwardLaunch& a, hipStream_t s);

// x = (T(raw) - dark) / norm over n pixels (dark / norm may be null).
hipError_t launch_correct(const void* raw, int32_t raw_dtype, const void* dark,
                          const void* norm, void* x, int32_t dtype, int64_t n,
                          hipStream_t s);

// norm = (flat * solid) * polar over the present arrays; returns false in
// *any when all three are null (norm untouched).
hipError_t launch_norm(const void* flat, const void* solid, const void* polar,
                       void* norm, int32_t dtype, int64_t n, hipStream_t s);

}  // namespace azi
