// Per-bin accumulators and reductions shared by the kernel translation
// units: double sums, or float sums with Kahan compensation (Section 5.2.2,
// merged across lanes with Knuth's TwoSum); the wavefront-level merge; the
// final write of W, U and I = W / U; the XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace azi {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Accumulators
// ---------------------------------------------------------------------------

struct AccF64 {
    using Slot = AccF64;  // what a partial-sum slot holds
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
    __device__ Slot slot() const { return *this; }
};

// W alone, for kernels whose U is taken from elsewhere (the folded
// coefficients carry 1 / norm, so their sums are not U): the same w
// operations as AccF64, and a partial-sum slot of AccF64's layout with u 0.
struct AccWF64 {
    using Slot = AccF64;
    double w;
    __device__ void zero() { w = 0.0; }
    template <class T>
    __device__ void add(T c, T x) { w = __fma_rn((double)c, (double)x, w); }
    __device__ void merge(const AccWF64& o) { w += o.w; }
    __device__ AccWF64 shfl_xor(int m) const {
        AccWF64 r;
        r.w = __shfl_xor(w, m, kWave);
        return r;
    }
    __device__ double W() const { return w; }
    __device__ double U() const { return 0.0; }
    __device__ Slot slot() const {
        Slot s;
        s.w = w;
        s.u = 0.0;
        return s;
    }
};

// Kahan (1965) compensated float sums; merge keeps the rounding error of the
// addition of the two leading parts (TwoSum) in the compensation term.
struct AccK32 {
    using Slot = AccK32;
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
    __device__ Slot slot() const { return *this; }
};

// The W half of AccK32 (see AccWF64).
struct AccWK32 {
    using Slot = AccK32;
    float ws, wc;
    __device__ void zero() { ws = wc = 0.0f; }
    template <class T>
    __device__ void add(T c, T x) { AccK32::kadd(ws, wc, __fmul_rn((float)c, (float)x)); }
    __device__ void merge(const AccWK32& o) {
        float s, e;
        AccK32::two_sum(ws, o.ws, s, e);
        wc = __fsub_rn(__fadd_rn(wc, o.wc), e);
        ws = s;
    }
    __device__ AccWK32 shfl_xor(int m) const {
        AccWK32 r;
        r.ws = __shfl_xor(ws, m, kWave);
        r.wc = __shfl_xor(wc, m, kWave);
        return r;
    }
    __device__ float W() const { return __fsub_rn(ws, wc); }
    __device__ float U() const { return 0.0f; }
    __device__ Slot slot() const {
        Slot s;
        s.ws = ws;
        s.wc = wc;
        s.us = 0.0f;
        s.uc = 0.0f;
        return s;
    }
};

// The W-only accumulator of an accumulator.
template <class Acc> struct WOnly;
template <> struct WOnly<AccF64> { using type = AccWF64; };
template <> struct WOnly<AccK32> { using type = AccWK32; };

static_assert(sizeof(AccF64) == 16 && sizeof(AccK32) == 16, "partial slot is 16 bytes");

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

// The plan's fixed per-bin terms of a reduction (see BandLaunch), loaded
// before the partial sums so that their latency overlaps them.
struct RowFixed {
    bool has_u = false, has_w = false;
    double u = 0.0, w = 0.0;
};

__device__ inline RowFixed load_row_fixed(int64_t r, const double* __restrict__ ufix_in,
                                          const double* __restrict__ wsub_in) {
    RowFixed f;
    if (ufix_in) {
        f.has_u = true;
        f.u = ufix_in[r];
        if (wsub_in) {
            f.has_w = true;
            f.w = wsub_in[r];
        }
    }
    return f;
}

// write_row with U taken from outside the partial sums (the plan's U in
// double) and a fixed term subtracted from W, or only U or W stored
// (ufix_out, wfix_out): see BandLaunch.
template <class T, class Acc>
__device__ inline void write_row_u(int32_t r, const Acc& a, T* __restrict__ I,
                                   T* __restrict__ W, T* __restrict__ U, double empty,
                                   const RowFixed& f, double* __restrict__ ufix_out,
                                   double* __restrict__ wfix_out) {
    if (ufix_out) {
        ufix_out[r] = (double)a.U();
        return;
    }
    if (wfix_out) {
        wfix_out[r] = (double)a.W();
        return;
    }
    if (!f.has_u) {
        write_row(r, a, I, W, U, empty);
        return;
    }
    using V = decltype(a.U());
    const V u = (V)f.u;
    V w = (V)a.W();
    if (f.has_w) w -= (V)f.w;
    if (W) W[r] = (T)w;
    if (U) U[r] = (T)u;
    I[r] = (u != 0) ? (T)(w / u) : (T)empty;
}

// Workgroup g runs on XCD g % 8; this maps it to a block index so that each
// XCD walks one contiguous eighth of the blocks (a bijection on [0, n)).
__device__ inline int64_t xcd_block(int64_t g, int64_t n) {
    if (n < 8) return g;
    const int64_t xcd = g & 7, q = g >> 3;
    const int64_t per = n >> 3, rem = n & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + q;
}

// One wavefront per bin adds the bin's partial sums (fixed lanes, fixed
// tree: deterministic) and writes W, U and I.
template <class T, class Acc>
__global__ void k_block_reduce(const int32_t* __restrict__ bin_ptr, int64_t b0, int64_t b1,
                               const Acc* __restrict__ parts, T* __restrict__ I,
                               T* __restrict__ W, T* __restrict__ U, double empty) {
    const int64_t b = b0 + (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (b >= b1) return;
    const int lane = threadIdx.x & (kWave - 1);
    Acc a;
    a.zero();
    for (int32_t k = bin_ptr[b] + lane; k < bin_ptr[b + 1]; k += kWave) a.merge(parts[k]);
    group_reduce(a, kWave);
    if (lane == 0) write_row((int32_t)b, a, I, W, U, empty);
}

}  // namespace
}  // namespace azi
