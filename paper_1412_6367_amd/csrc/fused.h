// Matrix-free integration kernel (host side): the bounding-box (or
// whole-pixel) coefficients of a planar orthogonal detector are recomputed
// per frame from the geometry instead of being read from a stored matrix.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace azi {

struct FusedLaunch {
    const FusedTile* tiles = nullptr;
    int32_t ntiles = 0;
    const int32_t* slots = nullptr;    // per tile, the slot of each bin of its window
    const int32_t* bin_ptr = nullptr;  // npt + 1
    azi_geom geom{};
    int32_t unit = AZI_UNIT_R_M;
    int32_t split = AZI_SPLIT_BBOX;    // AZI_SPLIT_BBOX or AZI_SPLIT_NONE
    double pmin = 0.0, delta = 1.0;
    int32_t npt = 0;
    const void* img = nullptr;         // image, element type img_dtype
    int32_t img_dtype = AZI_F64;
    const void* dark = nullptr;        // storage type, may be null
    const void* norm = nullptr;        // storage type, may be null
    void* parts = nullptr;             // 16 bytes per slot
    void* I = nullptr;
    void* W = nullptr;
    void* U = nullptr;
    double empty = 0.0;
    int32_t grid = 0;                  // 0: one workgroup per tile
    int32_t dtype = AZI_F64;
    int32_t accum = AZI_ACC_F64;
};

hipError_t launch_fused(const FusedLaunch& a, hipStream_t s);

}  // namespace azi
