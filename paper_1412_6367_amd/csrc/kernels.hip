// HIP kernels for gfx950 (CDNA4): the per-frame hot path of azimuthal
// integration.
//
//   k_spmv     gather-form sparse product of Section 5.2: every output bin
//              reads the pixels that feed it from the CSR (Section 5.2.1) and
//              forms W = sum c*x and U = sum c in one pass, then I = W / U.
//              Work is cut into tiles of bounded nonzero count (whole short
//              rows, or pieces of a long row); the sums of a piece go to a
//              partial slot and k_fixup adds the pieces of a row in order, so
//              results are deterministic and need no floating-point atomics.
//   k_fixup    finishes rows that were split over several tiles.
//   k_correct  cast + correction map of Section 6.4.
//   k_norm     (flat * solid) * polar, formed once per correction set.
//   k_prep_v / k_csc_bwd   adjoint: gx_p = sum_b A_bp (gI_b / U_b + gW_b),
//              one thread per pixel over its pixel-major (CSC) entries.
//
// Accumulation: double for either storage type (AZI_ACC_F64), or float with
// Kahan compensation (AZI_ACC_KAHAN32, Section 5.2.2), whose per-lane
// (sum, compensation) pairs are merged across lanes with Knuth's TwoSum.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace azi {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Accumulators
// ---------------------------------------------------------------------------

struct AccF64 {
    double w, u;
    __device__ void zero() { w = 0.0; u = 0.0; }
    template <class T>
    __device__ void add(T c, T x) {
        w = __fma_rn((double)c, (double)x, w);
        u += (double)c;
    }
    __device__ void merge(const AccF64& o) { w += o.w; u += o.u; }
    __device__ AccF64 shfl_xor(int m) const {
        AccF64 r;
        r.w = __shfl_xor(w, m, kWave);
        r.u = __shfl_xor(u, m, kWave);
        return r;
    }
    __device__ double W() const { return w; }
    __device__ double U() const { return u; }
};

// Kahan (1965) compensated float sums; merge keeps the rounding error of the
// addition of the two leading parts (TwoSum) in the compensation term.
struct AccK32 {
    float ws, wc, us, uc;  // running sum and compensation (to be added)
    __device__ void zero() { ws = wc = us = uc = 0.0f; }
    __device__ static void kadd(float& s, float& c, float v) {
        const float y = __fsub_rn(v, c);
        const float t = __fadd_rn(s, y);
        c = __fsub_rn(__fsub_rn(t, s), y);
        s = t;
    }
    __device__ static void two_sum(float a, float b, float& s, float& e) {
        s = __fadd_rn(a, b);
        const float bb = __fsub_rn(s, a);
        e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, bb)), __fsub_rn(b, bb));
    }
    template <class T>
    __device__ void add(T c, T x) {
        kadd(ws, wc, __fmul_rn((float)c, (float)x));
        kadd(us, uc, (float)c);
    }
    // Here wc / uc hold the amount ALREADY SUBTRACTED (Kahan's c): the value
    // of a pair is s - c.
    __device__ void merge(const AccK32& o) {
        float s, e;
        two_sum(ws, o.ws, s, e);
        wc = __fsub_rn(__fadd_rn(wc, o.wc), e);
        ws = s;
        two_sum(us, o.us, s, e);
        uc = __fsub_rn(__fadd_rn(uc, o.uc), e);
        us = s;
    }
    __device__ AccK32 shfl_xor(int m) const {
        AccK32 r;
        r.ws = __shfl_xor(ws, m, kWave);
        r.wc = __shfl_xor(wc, m, kWave);
        r.us = __shfl_xor(us, m, kWave);
        r.uc = __shfl_xor(uc, m, kWave);
        return r;
    }
    __device__ float W() const { return __fsub_rn(ws, wc); }
    __device__ float U() const { return __fsub_rn(us, uc); }
};

static_assert(sizeof(AccF64) == 16 && sizeof(AccK32) == 16, "partial slot is 16 bytes");

// ---------------------------------------------------------------------------
// Loads
// ---------------------------------------------------------------------------

__device__ inline void load4(const double* p, double v[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ inline void load4(const float* p, float v[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ inline void load4(const int32_t* p, int32_t v[4]) {
    const int4 a = *reinterpret_cast<const int4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Sums nonzeros [zlo, zhi) into `a`.  The `lanes` threads of a group (lane
// = 0 .. lanes-1) each take 4 consecutive nonzeros at a time from the
// 4-aligned window that covers the range; nonzeros outside the range are
// masked and their pixels are not read.  UNROLL windows are loaded before
// any of them is used, to keep that many requests in flight per lane.
template <int UNROLL, class T, class Acc>
__device__ inline void accumulate(Acc& a, int32_t zlo, int32_t zhi, int lane, int lanes,
                                  const int32_t* __restrict__ idx,
                                  const T* __restrict__ dat, const T* __restrict__ x) {
    const int32_t base = zlo & ~3;
    const int32_t step = 4 * lanes;
    for (int32_t z = base + 4 * lane; z < zhi; z += step * UNROLL) {
        int32_t iv[UNROLL][4];
        T dv[UNROLL][4];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t zz = z + u * step;
            if (zz < zhi) {
                load4(idx + zz, iv[u]);
                load4(dat + zz, dv[u]);
            }
        }
        T xv[UNROLL][4];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t zz = z + u * step;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int32_t e = zz + k;
                xv[u][k] = (e >= zlo && e < zhi) ? x[iv[u][k]] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t zz = z + u * step;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int32_t e = zz + k;
                if (e >= zlo && e < zhi) a.add(dv[u][k], xv[u][k]);
            }
        }
    }
}

template <class Acc>
__device__ inline void group_reduce(Acc& a, int lanes) {
    for (int m = lanes >> 1; m > 0; m >>= 1) a.merge(a.shfl_xor(m));
}

template <class T, class Acc>
__device__ inline void write_row(int32_t r, const Acc& a, T* __restrict__ I, T* __restrict__ W,
                                 T* __restrict__ U, double empty) {
    const auto w = a.W();
    const auto u = a.U();
    if (W) W[r] = (T)w;
    if (U) U[r] = (T)u;
    I[r] = (u != 0) ? (T)(w / u) : (T)empty;
}

template <class T, class Acc, int BLOCK, int UNROLL>
__device__ inline void process_tile(const Tile& t, Acc* red, const int32_t* __restrict__ rp,
                                    const int32_t* __restrict__ idx, const T* __restrict__ dat,
                                    const T* __restrict__ x, T* __restrict__ I,
                                    T* __restrict__ W, T* __restrict__ U,
                                    Acc* __restrict__ parts, double empty) {
    const int tid = threadIdx.x;
    const int32_t nr = t.r1 - t.r0;
    if (nr == 1) {
        // One row, or one piece of a long row: the whole workgroup sums it.
        Acc a;
        a.zero();
        accumulate<UNROLL>(a, t.z0, t.z1, tid, BLOCK, idx, dat, x);
        group_reduce(a, kWave);
        if ((tid & (kWave - 1)) == 0) red[tid / kWave] = a;
        __syncthreads();
        if (tid == 0) {
            Acc s = red[0];
            for (int k = 1; k < BLOCK / kWave; ++k) s.merge(red[k]);
            if (t.part < 0) write_row(t.r0, s, I, W, U, empty);
            else parts[t.part] = s;
        }
        __syncthreads();
        return;
    }
    // Several whole rows: a group of G lanes per row, G a power of two that
    // gives each lane about one 4-wide load per row, widened while the rows
    // cannot keep the workgroup busy.
    const int32_t avg = (t.z1 - t.z0 + nr - 1) / nr;
    int G = 1;
    while (G < kWave && 4 * G < avg) G <<= 1;
    while (G < kWave && nr * G < BLOCK) G <<= 1;
    const int ngroups = BLOCK / G;
    const int grp = tid / G;
    const int lane = tid & (G - 1);
    for (int32_t r = t.r0 + grp; r < t.r1; r += ngroups) {
        const int32_t q = t.ip0 + (r - t.r0);
        Acc a;
        a.zero();
        accumulate<UNROLL>(a, rp[q], rp[q + 1], lane, G, idx, dat, x);
        group_reduce(a, G);
        if (lane == 0) write_row(r, a, I, W, U, empty);
    }
}

// Tiles are visited XCD by XCD: the hardware deals consecutive workgroup ids
// to the 8 XCDs in turn, so workgroup g runs on XCD g % 8; giving that XCD a
// contiguous run of tiles keeps neighbouring bins -- which share most of
// their pixels -- in the same L2.
template <class T, class Acc, int BLOCK, int UNROLL>
__global__ __launch_bounds__(BLOCK) void k_spmv(const Tile* __restrict__ tiles, int32_t ntiles,
                                                const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ idx,
                                                const T* __restrict__ dat,
                                                const T* __restrict__ x, T* __restrict__ I,
                                                T* __restrict__ W, T* __restrict__ U,
                                                Acc* __restrict__ parts, double empty) {
    __shared__ Acc red[BLOCK / kWave];
    const int32_t g = blockIdx.x, G = gridDim.x;
    if (G < 8) {
        for (int32_t t = g; t < ntiles; t += G)
            process_tile<T, Acc, BLOCK, UNROLL>(tiles[t], red, rp, idx, dat, x, I, W, U, parts, empty);
        return;
    }
    const int32_t xcd = g & 7, q = g >> 3;
    const int32_t nq = (G - xcd + 7) >> 3;
    const int32_t per = ntiles >> 3, rem = ntiles & 7;
    const int32_t t0 = xcd * per + min(xcd, rem);
    const int32_t t1 = t0 + per + (xcd < rem ? 1 : 0);
    for (int32_t t = t0 + q; t < t1; t += nq)
        process_tile<T, Acc, BLOCK, UNROLL>(tiles[t], red, rp, idx, dat, x, I, W, U, parts, empty);
}

template <class T, class Acc>
__global__ void k_fixup(const Split* __restrict__ splits, int32_t nsplits,
                        const Acc* __restrict__ parts, T* __restrict__ I, T* __restrict__ W,
                        T* __restrict__ U, double empty) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsplits) return;
    const Split s = splits[k];
    Acc a = parts[s.p0];
    for (int32_t p = s.p0 + 1; p < s.p1; ++p) a.merge(parts[p]);
    write_row(s.row, a, I, W, U, empty);
}

// ---------------------------------------------------------------------------
// Correction map (Section 6.4)
// ---------------------------------------------------------------------------

template <class R, class T>
__global__ void k_correct(const R* __restrict__ raw, const T* __restrict__ dark,
                          const T* __restrict__ norm, T* __restrict__ x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        T v = (T)raw[i];
        if (dark) v = v - dark[i];
        if (norm) v = v / norm[i];
        x[i] = v;
    }
}

template <class T>
__global__ void k_norm(const T* __restrict__ a, const T* __restrict__ b, const T* __restrict__ c,
                       T* __restrict__ norm, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        bool have = false;
        T v = T(1);
        if (a) { v = a[i]; have = true; }
        if (b) { v = have ? v * b[i] : b[i]; have = true; }
        if (c) { v = have ? v * c[i] : c[i]; }
        norm[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_prep_v(const T* __restrict__ U, const T* __restrict__ gI,
                         const T* __restrict__ gW, double* __restrict__ v, int64_t n) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double val = 0.0;
    if (gI) {
        const double u = (double)U[b];
        val = (u != 0.0) ? (double)gI[b] / u : 0.0;
    }
    if (gW) val = val + (double)gW[b];
    v[b] = val;
}

template <class T>
__global__ void k_csc_bwd(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                          const T* __restrict__ cdata, const double* __restrict__ v,
                          const T* __restrict__ norm, T* __restrict__ gx, int64_t npix) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        const int32_t k0 = colptr[p], k1 = colptr[p + 1];
        double acc = 0.0;
        for (int32_t k = k0; k < k1; ++k) acc = __fma_rn((double)cdata[k], v[rowidx[k]], acc);
        if (norm) acc = acc / (double)norm[p];
        gx[p] = (T)acc;
    }
}

int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

template <class T, class Acc, int BLOCK>
hipError_t forward_impl(const ForwardLaunch& a, hipStream_t s) {
    constexpr int UNROLL = 2;
    if (a.ntiles > 0) {
        const int grid = a.grid > 0 ? a.grid : a.ntiles;
        hipLaunchKernelGGL((k_spmv<T, Acc, BLOCK, UNROLL>), dim3(grid), dim3(BLOCK), 0, s,
                           a.tiles, a.ntiles, a.rowptr, a.indices,
                           static_cast<const T*>(a.data), static_cast<const T*>(a.x),
                           static_cast<T*>(a.I), static_cast<T*>(a.W), static_cast<T*>(a.U),
                           static_cast<Acc*>(a.parts), a.empty);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.nsplits > 0) {
        hipLaunchKernelGGL((k_fixup<T, Acc>), dim3(grid_for(a.nsplits, 256)), dim3(256), 0, s,
                           a.splits, a.nsplits, static_cast<const Acc*>(a.parts),
                           static_cast<T*>(a.I), static_cast<T*>(a.W), static_cast<T*>(a.U),
                           a.empty);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <class T, class Acc>
hipError_t forward_block(const ForwardLaunch& a, hipStream_t s) {
    switch (a.block) {
        case 64: return forward_impl<T, Acc, 64>(a, s);
        case 128: return forward_impl<T, Acc, 128>(a, s);
        case 256: return forward_impl<T, Acc, 256>(a, s);
        case 512: return forward_impl<T, Acc, 512>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class R, class T>
hipError_t correct_impl(const void* raw, const void* dark, const void* norm, void* x, int64_t n,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_correct<R, T>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<const R*>(raw), static_cast<const T*>(dark),
                       static_cast<const T*>(norm), static_cast<T*>(x), n);
    return hipGetLastError();
}

template <class T>
hipError_t correct_raw(const void* raw, int32_t raw_dtype, const void* dark, const void* norm,
                       void* x, int64_t n, hipStream_t s) {
    switch (raw_dtype) {
        case AZI_I16: return correct_impl<int16_t, T>(raw, dark, norm, x, n, s);
        case AZI_U16: return correct_impl<uint16_t, T>(raw, dark, norm, x, n, s);
        case AZI_I32: return correct_impl<int32_t, T>(raw, dark, norm, x, n, s);
        case AZI_U32: return correct_impl<uint32_t, T>(raw, dark, norm, x, n, s);
        case AZI_F32: return correct_impl<float, T>(raw, dark, norm, x, n, s);
        case AZI_F64: return correct_impl<double, T>(raw, dark, norm, x, n, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T>
hipError_t backward_impl(const BackwardLaunch& a, hipStream_t s) {
    if (a.npt > 0) {
        hipLaunchKernelGGL((k_prep_v<T>), dim3((unsigned)((a.npt + 255) / 256)), dim3(256), 0, s,
                           static_cast<const T*>(a.U), static_cast<const T*>(a.gI),
                           static_cast<const T*>(a.gW), a.v, a.npt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.npix > 0) {
        hipLaunchKernelGGL((k_csc_bwd<T>), dim3(grid_for(a.npix, 256)), dim3(256), 0, s,
                           a.colptr, a.rowidx, static_cast<const T*>(a.cdata), a.v,
                           static_cast<const T*>(a.norm), static_cast<T*>(a.gx), a.npix);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_forward(const ForwardLaunch& a, hipStream_t s) {
    if (a.dtype == AZI_F64) return forward_block<double, AccF64>(a, s);
    if (a.accum == AZI_ACC_KAHAN32) return forward_block<float, AccK32>(a, s);
    return forward_block<float, AccF64>(a, s);
}

hipError_t launch_backward(const BackwardLaunch& a, hipStream_t s) {
    return a.dtype == AZI_F64 ? backward_impl<double>(a, s) : backward_impl<float>(a, s);
}

hipError_t launch_correct(const void* raw, int32_t raw_dtype, const void* dark, const void* norm,
                          void* x, int32_t dtype, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return dtype == AZI_F64 ? correct_raw<double>(raw, raw_dtype, dark, norm, x, n, s)
                            : correct_raw<float>(raw, raw_dtype, dark, norm, x, n, s);
}

hipError_t launch_norm(const void* flat, const void* solid, const void* polar, void* norm,
                       int32_t dtype, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dtype == AZI_F64) {
        hipLaunchKernelGGL((k_norm<double>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                           static_cast<const double*>(flat), static_cast<const double*>(solid),
                           static_cast<const double*>(polar), static_cast<double*>(norm), n);
    } else {
        hipLaunchKernelGGL((k_norm<float>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                           static_cast<const float*>(flat), static_cast<const float*>(solid),
                           static_cast<const float*>(polar), static_cast<float*>(norm), n);
    }
    return hipGetLastError();
}

}  // namespace azi
