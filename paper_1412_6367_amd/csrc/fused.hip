// Matrix-free integration: per frame, every image tile recomputes its
// pixels' radial extents and bounding-box shares (Section 4.1) from the
// planar geometry -- the same IEEE operations as the plan builders, this
// translation unit being compiled without contraction like them -- so the
// only data streamed from HBM is the image itself, plus a partial sum per
// (tile, bin).  Deterministic: every bin's partial is summed in a fixed
// order, no floating-point atomics.
//
// Phase 1: one thread per pixel stores the cast and corrected value and its
//   bin range [b0, b1] with the three distinct shares (first, inner, last)
//   in LDS.
// Phase 2: along an image row the pixels on each side of the beam column
//   have radial extents that grow monotonically away from it, so the pixels
//   feeding bin b form one contiguous run per side.  A table per row gives
//   the first pixel of that run (filled race-free: each bin by the one pixel
//   where the running last bin passes it).  A wavefront takes 64 / rows bins
//   at a time, one lane per (bin, tile row): each lane walks its row's runs, left
//   side then right side, and the row sums of a bin are merged by a fixed
//   shuffle tree and written to the bin's slot; k_block_reduce adds the
//   slots of each bin in tile order.
#include "fused.h"

#include "accum.h"
#include "pixel_math.h"

namespace azi {
namespace {

constexpr int kFB = 256;                   // threads per workgroup
constexpr int kFPix = kFusedH * kFusedW;   // pixels per tile
constexpr int kPitch = kFusedW + 1;        // LDS row pitch: rows of a column in distinct banks
constexpr int kLdsPix = kFusedH * kPitch;
constexpr int kFWin = 128;                 // bins per pass over a tile
constexpr int kTPitch = kFWin + 4;         // table row pitch (bytes), same reason
constexpr int kBinsPerWave = kWave / kFusedH;
constexpr int32_t kBig = 1 << 30;          // bin of pixels outside the range
static_assert(kFusedW <= 127, "column index kept in int8");
static_assert(kWave % kFusedH == 0, "a wavefront holds whole bins");

// Output coordinate of a radius: the plan builder's to_unit; kTrig false
// compiles only the radial units (no atan / sin code, fewer registers).
template <bool kTrig>
__device__ inline double unit_of(double r, int32_t unit, const azi_geom& g) {
    if constexpr (kTrig) return to_unit(r, unit, g.dist_m, g.wavelength_m);
    else return unit == AZI_UNIT_R_MM ? r * 1e3 : r;
}

template <class R, class T, class Acc, bool kTrig>
__global__ __launch_bounds__(kFB) void k_fused(const FusedTile* __restrict__ tiles,
                                               int32_t ntiles, const int32_t* __restrict__ slots,
                                               azi_geom g, int32_t unit, int32_t split,
                                               double pmin, double delta, int32_t npt,
                                               const R* __restrict__ img,
                                               const T* __restrict__ dark,
                                               const T* __restrict__ norm,
                                               Acc* __restrict__ parts) {
    __shared__ T xs[kLdsPix];
    __shared__ T cls[kLdsPix], cis[kLdsPix], crs[kLdsPix];
    __shared__ int32_t b0s[kLdsPix], b1s[kLdsPix];
    __shared__ int8_t first_r[kFusedH][kTPitch], first_l[kFusedH][kTPitch];
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    const int row = lane % kFusedH, sub = lane / kFusedH;
    const int32_t gi = blockIdx.x, Gd = gridDim.x;
    int32_t t_begin, t_end, t_step;
    if (Gd < 8) {
        t_begin = gi; t_end = ntiles; t_step = Gd;
    } else {
        const int32_t xcd = gi & 7, q = gi >> 3, nq = (Gd - xcd + 7) >> 3;
        const int32_t per = ntiles >> 3, rem = ntiles & 7;
        const int32_t t0 = xcd * per + min(xcd, rem);
        t_begin = t0 + q; t_end = t0 + per + (xcd < rem ? 1 : 0); t_step = nq;
    }
    const double beam_col = ::floor(g.center_x_px);
    for (int32_t ti = t_begin; ti < t_end; ti += t_step) {
        const FusedTile t = tiles[ti];
        if (t.nwin == 0) continue;  // uniform over the workgroup
        // phase 1: values and shares (one pixel at a time per thread keeps
        // the double-precision square roots and divisions in few registers)
#pragma unroll 1
        for (int e = tid; e < kFPix; e += kFB) {
            const int r = e / kFusedW, c = e - r * kFusedW;
            int32_t b0 = kBig, b1 = kBig;
            T cl = T(0), ci = T(0), cr = T(0), xv = T(0);
            if (r < t.th && c < t.tw) {
                const int64_t i = t.i0 + r, j = t.j0 + c;
                const int64_t p = i * g.w + j;
                T v = (T)img[p];
                if (dark) v = v - dark[p];
                if (norm) v = v / norm[p];
                xv = v;
                const Extent ex = pixel_extent(i, j, g);
                if (split == AZI_SPLIT_NONE) {
                    const double fc = (unit_of<kTrig>(ex.mid, unit, g) - pmin) / delta;
                    if (fc >= 0.0 && fc <= (double)npt) {
                        b0 = b1 = vmin((int32_t)::floor(fc), npt - 1);
                        cl = T(1);
                    } else {
                        b0 = b1 = fc < 0.0 ? -kBig : kBig;
                    }
                } else {
                    const BoxTerms bt = bbox_terms(unit_of<kTrig>(ex.lo, unit, g),
                                                   unit_of<kTrig>(ex.hi, unit, g), pmin, delta,
                                                   npt);
                    if (bt.b0 > bt.b1) {
                        b0 = b1 = bt.fl >= (double)npt ? kBig : -kBig;
                    } else {
                        b0 = bt.b0;
                        b1 = bt.b1;
                        cl = (T)bt.cl;
                        ci = (T)bt.ci;
                        cr = (T)bt.cr;
                    }
                }
            }
            const int l = r * kPitch + c;
            xs[l] = xv;
            cls[l] = cl;
            cis[l] = ci;
            crs[l] = cr;
            b0s[l] = b0;
            b1s[l] = b1;
        }
        // columns [0, cs) lie left of the beam column, [cs, tw) right of it
        const int cs = (int)vmin(vmax(beam_col - (double)t.j0, 0.0), (double)t.tw);
        for (int32_t w0 = t.wlo; w0 < t.wlo + t.nwin; w0 += kFWin) {
            const int32_t nw = min(kFWin, t.wlo + t.nwin - w0);
            const int32_t w1 = w0 + nw - 1;
            for (int e = tid; e < kFusedH * kTPitch; e += kFB) {
                first_r[e / kTPitch][e % kTPitch] = -1;
                first_l[e / kTPitch][e % kTPitch] = -1;
            }
            __syncthreads();
            // each bin is claimed by the pixel of the run where the running
            // last bin first reaches it
            for (int e = tid; e < kFPix; e += kFB) {
                const int r = e / kFusedW, c = e - r * kFusedW;
                if (r >= t.th || c >= t.tw) continue;
                const int l = r * kPitch + c;
                const bool right = c >= cs;
                const bool first = right ? c == cs : c == cs - 1;
                const int32_t prev = first ? -kBig : b1s[right ? l - 1 : l + 1];
                const int32_t lo_b = max(prev + 1, w0);
                const int32_t hi_b = min(b1s[l], w1);
                for (int32_t b = lo_b; b <= hi_b; ++b) {
                    if (right) first_r[r][b - w0] = (int8_t)c;
                    else first_l[r][b - w0] = (int8_t)c;
                }
            }
            __syncthreads();
            // phase 2: one lane per (bin, row); four bins per wavefront pass
            for (int32_t q0 = wave * kBinsPerWave; q0 < nw; q0 += (kFB / kWave) * kBinsPerWave) {
                const int32_t q = q0 + sub;
                Acc a;
                a.zero();
                if (q < nw && row < t.th) {
                    const int32_t b = w0 + q;
                    for (int c = first_l[row][q]; c >= 0; --c) {
                        const int e = row * kPitch + c;
                        if (b0s[e] > b) break;
                        const T cv = b == b0s[e] ? cls[e] : (b == b1s[e] ? crs[e] : cis[e]);
                        a.add(cv, xs[e]);
                    }
                    const int c0 = first_r[row][q];
                    if (c0 >= 0) {
                        for (int c = c0; c < t.tw; ++c) {
                            const int e = row * kPitch + c;
                            if (b0s[e] > b) break;
                            const T cv = b == b0s[e] ? cls[e] : (b == b1s[e] ? crs[e] : cis[e]);
                            a.add(cv, xs[e]);
                        }
                    }
                }
                group_reduce(a, kFusedH);
                if (row == 0 && q < nw) parts[slots[t.slot_off + (w0 - t.wlo) + q]] = a;
            }
            __syncthreads();
        }
    }
}

template <class R, class T, class Acc>
hipError_t run(const FusedLaunch& a, hipStream_t s) {
    const int32_t grid = a.grid > 0 ? min(a.grid, a.ntiles) : a.ntiles;
    const bool trig = a.unit != AZI_UNIT_R_M && a.unit != AZI_UNIT_R_MM;
    if (a.ntiles > 0) {
        if (trig)
            hipLaunchKernelGGL((k_fused<R, T, Acc, true>), dim3((unsigned)grid), dim3(kFB), 0, s,
                               a.tiles, a.ntiles, a.slots, a.geom, a.unit, a.split, a.pmin,
                               a.delta, a.npt, static_cast<const R*>(a.img),
                               static_cast<const T*>(a.dark), static_cast<const T*>(a.norm),
                               static_cast<Acc*>(a.parts));
        else
            hipLaunchKernelGGL((k_fused<R, T, Acc, false>), dim3((unsigned)grid), dim3(kFB), 0, s,
                               a.tiles, a.ntiles, a.slots, a.geom, a.unit, a.split, a.pmin,
                               a.delta, a.npt, static_cast<const R*>(a.img),
                               static_cast<const T*>(a.dark), static_cast<const T*>(a.norm),
                               static_cast<Acc*>(a.parts));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.npt > 0) {
        const int64_t blocks = ((int64_t)a.npt + 3) / 4;  // 4 wavefronts per 256 threads
        hipLaunchKernelGGL((k_block_reduce<T, Acc>), dim3((unsigned)blocks), dim3(256), 0, s,
                           a.bin_ptr, (int64_t)0, (int64_t)a.npt, static_cast<const Acc*>(a.parts),
                           static_cast<T*>(a.I), static_cast<T*>(a.W), static_cast<T*>(a.U),
                           a.empty);
    }
    return hipGetLastError();
}

template <class T, class Acc>
hipError_t by_image(const FusedLaunch& a, hipStream_t s) {
    switch (a.img_dtype) {
        case AZI_I16: return run<int16_t, T, Acc>(a, s);
        case AZI_U16: return run<uint16_t, T, Acc>(a, s);
        case AZI_I32: return run<int32_t, T, Acc>(a, s);
        case AZI_U32: return run<uint32_t, T, Acc>(a, s);
        case AZI_F32: return run<float, T, Acc>(a, s);
        case AZI_F64: return run<double, T, Acc>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fused(const FusedLaunch& a, hipStream_t s) {
    if (a.split != AZI_SPLIT_BBOX && a.split != AZI_SPLIT_NONE) return hipErrorInvalidValue;
    if (a.dtype == AZI_F64) return by_image<double, AccF64>(a, s);
    if (a.accum == AZI_ACC_KAHAN32) return by_image<float, AccK32>(a, s);
    return by_image<float, AccF64>(a, s);
}

}  // namespace azi
