// HIP kernels for gfx950 (CDNA4): the per-frame hot path of azimuthal
// integration.
//
//   k_band_runs  the default integration (run layout): bands of 4 bins
//              whose entries are ordered by pixel, stored as one word per
//              run of a pixel's entries in the band, so a wavefront gathers
//              nearly consecutive pixels of the row-major image once per run;
//              lane-private accumulators per band row; the partial sums of
//              each piece go to slots that k_band_reduce adds in piece order.
//              Its raw-frame form casts and corrects every pixel it gathers.
//   k_band     the same over one word per entry (band layout, R = 4, 8, 16).
//   k_spmv     gather-form sparse product of Section 5.2 on the CSR of
//              Section 5.2.1 (pixel and ring layouts): every output bin
//              reads the pixels that feed it and forms W = sum c*x and
//              U = sum c in one pass, then I = W / U.  Work is cut into tiles
//              of bounded nonzero count (whole short rows, or pieces of a
//              long row); k_fixup adds the pieces of a row in order.
//   k_block    the tile layout: image tiles staged in LDS, per-(tile, bin)
//              partials added by k_block_reduce.
//   k_correct  cast + correction map of Section 6.4; k_stage_* the same
//              into ring order; k_norm (flat * solid) * polar and
//              k_corr_pair (dark, 1 / norm) or k_corr_record12, formed once
//              per correction set.
//   k_prep_v / k_csc_bwd   adjoint: gx_p = sum_b A_bp (gI_b / U_b + gW_b),
//              one thread per pixel over its pixel-major (CSC) entries.
//
// Every sum has a fixed order (no floating-point atomics).  Accumulation:
// double for either storage type (AZI_ACC_F64), or float with Kahan
// compensation (AZI_ACC_KAHAN32, Section 5.2.2), whose per-lane (sum,
// compensation) pairs are merged across lanes with Knuth's TwoSum.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "accum.h"
#include "kernels.h"

namespace azi {
namespace {

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

template <bool NT, class T>
__device__ inline T ld(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Lane-strided form: lane j of the group takes nonzeros zlo + j, + lanes, ...
// so one gather instruction reads `lanes` consecutive nonzeros of a row --
// pixels that sit next to each other on the detector -- and touches few
// cache lines.  NT_IDX / NT_DAT stream the pixel ids / coefficients with
// non-temporal loads, leaving the caches to the image being gathered.
template <int UNROLL, bool NT_IDX, bool NT_DAT, class T, class Acc>
__device__ inline void accumulate_strided(Acc& a, int32_t zlo, int32_t zhi, int lane, int lanes,
                                          const int32_t* __restrict__ idx,
                                          const T* __restrict__ dat, const T* __restrict__ x) {
    for (int32_t z = zlo + lane; z < zhi; z += lanes * UNROLL) {
        int32_t iv[UNROLL];
        T dv[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t e = z + u * lanes;
            if (e < zhi) {
                iv[u] = ld<NT_IDX>(idx + e);
                dv[u] = ld<NT_DAT>(dat + e);
            }
        }
        T xv[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) xv[u] = (z + u * lanes < zhi) ? x[iv[u]] : T(0);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            if (z + u * lanes < zhi) a.add(dv[u], xv[u]);
    }
}

// Kernel variants (load layout, unroll depth, non-temporal pixel ids /
// coefficients).  Variant 2 keeps the pixel ids cached and streams the
// coefficients: for the short rows of 2-D plans the ids stay in the
// last-level cache from frame to frame while the coefficients would evict
// the gathered pixels.
template <int VAR> struct Variant;
template <> struct Variant<0> { static constexpr bool x4 = true;  static constexpr int unroll = 2; static constexpr bool nt_idx = false, nt_dat = false; };
template <> struct Variant<1> { static constexpr bool x4 = false; static constexpr int unroll = 4; static constexpr bool nt_idx = false, nt_dat = false; };
template <> struct Variant<2> { static constexpr bool x4 = false; static constexpr int unroll = 8; static constexpr bool nt_idx = false, nt_dat = true; };
template <> struct Variant<3> { static constexpr bool x4 = false; static constexpr int unroll = 8; static constexpr bool nt_idx = true, nt_dat = true; };
template <> struct Variant<4> { static constexpr bool x4 = true;  static constexpr int unroll = 4; static constexpr bool nt_idx = false, nt_dat = false; };
template <> struct Variant<5> { static constexpr bool x4 = false; static constexpr int unroll = 16; static constexpr bool nt_idx = true, nt_dat = true; };
template <> struct Variant<6> { static constexpr bool x4 = false; static constexpr int unroll = 16; static constexpr bool nt_idx = false, nt_dat = false; };
constexpr int kVariants = 7;

template <int VAR, class T, class Acc>
__device__ inline void accumulate_var(Acc& a, int32_t zlo, int32_t zhi, int lane, int lanes,
                                      const int32_t* __restrict__ idx, const T* __restrict__ dat,
                                      const T* __restrict__ x) {
    using V = Variant<VAR>;
    if constexpr (V::x4) accumulate<V::unroll>(a, zlo, zhi, lane, lanes, idx, dat, x);
    else accumulate_strided<V::unroll, V::nt_idx, V::nt_dat>(a, zlo, zhi, lane, lanes, idx, dat, x);
}

template <class T, class Acc, int BLOCK, int VAR>
__device__ inline void process_tile(const Tile& t, Acc* red, const int32_t* __restrict__ rp,
                                    const int32_t* __restrict__ idx, const T* __restrict__ dat,
                                    const T* __restrict__ x, T* __restrict__ I,
                                    T* __restrict__ W, T* __restrict__ U,
                                    Acc* __restrict__ parts, double empty) {
    const int tid = threadIdx.x;
    const int32_t nr = t.r1 - t.r0;
    if (t.mode == kTileRow) {
        // One row, or one piece of a long row: the whole workgroup sums it.
        Acc a;
        a.zero();
        accumulate_var<VAR>(a, t.z0, t.z1, tid, BLOCK, idx, dat, x);
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
    int G = 1;
    if (t.mode == kTileInterleave) {
        // every row gets BLOCK / nr lanes (a power of two, at most a wave)
        while (G < kWave && 2 * G * nr <= BLOCK) G <<= 1;
    } else {
        // whole rows: about one 4-wide load per lane and row, widened while
        // the rows cannot keep the workgroup busy
        const int32_t avg = (t.z1 - t.z0 + nr - 1) / nr;
        while (G < kWave && 4 * G < avg) G <<= 1;
        while (G < kWave && nr * G < BLOCK) G <<= 1;
    }
    const int ngroups = BLOCK / G;
    const int grp = tid / G;
    const int lane = tid & (G - 1);
    for (int32_t i = grp; i < nr; i += ngroups) {
        const int32_t q = t.ip0 + i;
        int32_t zlo = rp[q], zhi = rp[q + 1];
        if (t.mode == kTileInterleave) {
            const int32_t a0 = zlo, b0 = zhi;
            zlo = piece_cut(a0, b0, t.k, t.z1);
            zhi = piece_cut(a0, b0, t.k + 1, t.z1);
        }
        Acc a;
        a.zero();
        accumulate_var<VAR>(a, zlo, zhi, lane, G, idx, dat, x);
        group_reduce(a, G);
        if (lane == 0) {
            if (t.mode == kTileInterleave && t.part >= 0) parts[t.part + i * t.z1 + t.k] = a;
            else write_row(t.r0 + i, a, I, W, U, empty);
        }
    }
}

// Tiles are visited XCD by XCD: the hardware deals consecutive workgroup ids
// to the 8 XCDs in turn, so workgroup g runs on XCD g % 8; giving that XCD a
// contiguous run of tiles keeps neighbouring bins -- which share most of
// their pixels -- in the same L2.
template <class T, class Acc, int BLOCK, int VAR>
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
            process_tile<T, Acc, BLOCK, VAR>(tiles[t], red, rp, idx, dat, x, I, W, U, parts, empty);
        return;
    }
    const int32_t xcd = g & 7, q = g >> 3;
    const int32_t nq = (G - xcd + 7) >> 3;
    const int32_t per = ntiles >> 3, rem = ntiles & 7;
    const int32_t t0 = xcd * per + min(xcd, rem);
    const int32_t t1 = t0 + per + (xcd < rem ? 1 : 0);
    for (int32_t t = t0 + q; t < t1; t += nq)
        process_tile<T, Acc, BLOCK, VAR>(tiles[t], red, rp, idx, dat, x, I, W, U, parts, empty);
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
// Band form: entries of R consecutive bins ordered by pixel id
// ---------------------------------------------------------------------------

// One workgroup per piece of a band.  Lanes take consecutive entries (one
// coalesced load of packed ids and coefficients per instruction; the pixels
// they gather are nearly consecutive in the row-major image) and add each
// product to the accumulator of the entry's bin within the band.  The R
// accumulators are then reduced over the workgroup in a fixed tree and
// written to the piece's R partial slots.
template <class T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// (T(raw) - dark) * (1 / norm) from a pair of the storage type, or from a
// 12-byte record (float dark, double 1 / norm) used when every dark value
// is a float: the cast back to double is exact, so both give the same bits.
__device__ inline double corr_apply(double v, const double2& c) { return (v - c.x) * c.y; }
__device__ inline float corr_apply(float v, const float2& c) { return (v - c.x) * c.y; }
__device__ inline double corr_apply(double v, const Corr12& c) {
    const double inv = __hiloint2double((int)c.inv_hi, (int)c.inv_lo);
    return (v - (double)c.dark) * inv;
}
// Dark alone, when the coefficients carry 1 / norm (AZI_STAGE_FOLD): the
// difference of an integer count and a float dark is exact in double.
__device__ inline double corr_apply(double v, float d) { return v - (double)d; }
__device__ inline double corr_apply(double v, double d) { return v - d; }
__device__ inline float corr_apply(float v, float d) { return v - d; }
// An integer dark count of 16 bits: exact in float and double alike.
__device__ inline double corr_apply(double v, uint16_t d) { return v - (double)d; }
__device__ inline float corr_apply(float v, uint16_t d) { return v - (float)d; }
template <class T, class V>
__device__ inline T corr_apply(T v, RunDark<V> d) { return corr_apply(v, d.v); }
template <class C> struct IsRunDark { static constexpr bool value = false; };
template <class V> struct IsRunDark<RunDark<V>> { static constexpr bool value = true; };

// With kCorr the image is the raw frame: every gathered pixel is cast and
// corrected on the way, (T(raw) - dark) * (1 / norm), dark and the
// reciprocal of norm coming as one pair per pixel (one load), so the
// corrected image is never written.
template <class T, class Acc, int BLOCK, int R, class RawT = T, bool kCorr = false,
          class CorrT = typename Pair2<T>::type>
__global__ __launch_bounds__(BLOCK) void k_band(const BandPiece* __restrict__ pieces,
                                                int32_t npieces,
                                                const int32_t* __restrict__ packed,
                                                const T* __restrict__ coef,
                                                const T* __restrict__ x,
                                                Acc* __restrict__ parts,
                                                const RawT* __restrict__ raw = nullptr,
                                                const CorrT* __restrict__ corr = nullptr) {
    constexpr int U = 4;
    constexpr int32_t kMask = (1 << kBandShift) - 1;
    __shared__ Acc red[BLOCK / kWave][R];
    const int tid = threadIdx.x;
    const int32_t g = blockIdx.x, Gd = gridDim.x;
    int32_t t_begin, t_end, t_step;
    if (Gd < 8) {
        t_begin = g; t_end = npieces; t_step = Gd;
    } else {
        const int32_t xcd = g & 7, q = g >> 3, nq = (Gd - xcd + 7) >> 3;
        const int32_t per = npieces >> 3, rem = npieces & 7;
        const int32_t t0 = xcd * per + min(xcd, rem);
        t_begin = t0 + q; t_end = t0 + per + (xcd < rem ? 1 : 0); t_step = nq;
    }
    for (int32_t ti = t_begin; ti < t_end; ti += t_step) {
        const BandPiece pc = pieces[ti];
        const T* xb = kCorr ? nullptr : x + pc.pix_off;
        const RawT* rb = kCorr ? raw + pc.pix_off : nullptr;
        const CorrT* cb = (kCorr && corr) ? corr + pc.pix_off : nullptr;
        Acc a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r].zero();
        for (int32_t z = pc.z0 + tid; z < pc.z1; z += BLOCK * U) {
            int32_t pk[U];
            T cv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t zz = z + u * BLOCK;
                if (zz < pc.z1) {
                    pk[u] = __builtin_nontemporal_load(packed + zz);
                    cv[u] = __builtin_nontemporal_load(coef + zz);
                }
            }
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (kCorr) {
                    T v = T(0);
                    if (z + u * BLOCK < pc.z1) {
                        const int32_t pix = pk[u] & kMask;
                        v = (T)rb[pix];
                        if (cb) v = corr_apply(v, cb[pix]);
                    }
                    xv[u] = v;
                } else {
                    xv[u] = (z + u * BLOCK < pc.z1) ? xb[pk[u] & kMask] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (z + u * BLOCK < pc.z1) {
                    const int row = pk[u] >> kBandShift;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == row) a[r].add(cv[u], xv[u]);
                }
            }
        }
        const int wave = tid / kWave, lane = tid & (kWave - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            group_reduce(a[r], kWave);
            if (lane == 0) red[wave][r] = a[r];
        }
        __syncthreads();
        if (tid < R) {
            Acc sacc = red[0][tid];
            for (int k = 1; k < BLOCK / kWave; ++k) sacc.merge(red[k][tid]);
            parts[pc.slot0 + tid] = sacc;
        }
        __syncthreads();
    }
}

// Run encoding of the band layout: a wavefront takes a group of 64 runs
// (lane = run), reads each run's word, finds where its 1..4 coefficients
// sit from the group's counts (ballots and lane ranks: no table), gathers
// the pixel once for the whole run and adds each coefficient's product to
// the accumulator of its row.  run_groups handles U such groups at once,
// the u-th starting at run z + u * stride (none at or beyond z1).
template <class T, class Acc, int U, class RawT, bool kCorr, class CorrT>
__device__ __forceinline__ void run_groups(int32_t z, int32_t stride, int32_t z1, int lane,
                                           const int32_t* __restrict__ runs,
                                           const int32_t* __restrict__ gbase,
                                           const T* __restrict__ coef, const T* __restrict__ x,
                                           const RawT* __restrict__ raw,
                                           const CorrT* __restrict__ corr, int64_t pix_off,
                                           Acc (&a)[kRunRows]) {
    constexpr int R = kRunRows;
    constexpr int32_t kMask = (1 << kBandShift) - 1;
    constexpr bool kRunCorr = kCorr && IsRunDark<CorrT>::value;
    // Float64 streams the run words, per-run dark values and coefficients
    // non-temporally; float32 keeps them in the caches (c2 frame, folded
    // step, back to back / flushed: float32 64-65 / 71 us cached against 71
    // / 73 us streamed; float64 with the words and darks cached 82 / 91 us
    // against 88 / 90 us, and the 4096-image float64 batch 6 % slower).
    constexpr bool kNt = sizeof(T) == 8;
    int32_t rw[U], base[U];
    CorrT dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t zg = z + u * stride;       // uniform over the wavefront
        rw[u] = -1;
        base[u] = 0;
        if (zg < z1) {
            base[u] = gbase[zg >> 6];
            if (zg + lane < z1) {
                rw[u] = ld<kNt>(runs + zg + lane);
                if constexpr (kRunCorr) {
                    if (corr)
                        dv[u].v = ld<kNt>(reinterpret_cast<const decltype(dv[u].v)*>(corr) + zg +
                                          lane);
                }
            }
        }
    }
    T c[U][R];
    int n[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        n[u] = rw[u] < 0 ? 0 : ((rw[u] >> kRunCountShift) & 3) + 1;
        int32_t off = base[u];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const uint64_t m = __ballot(n[u] > j);
            const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            c[u][j] = n[u] > j ? ld<kNt>(coef + off + rank) : T(0);
            off += (int32_t)__popcll(m);
        }
    }
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        T v = T(0);
        if (n[u] > 0) {
            const int32_t pix = rw[u] & kMask;
            if constexpr (kRunCorr) {
                v = (T)raw[pix_off + pix];
                if (corr) v = corr_apply(v, dv[u]);
            } else if constexpr (kCorr) {
                v = (T)raw[pix_off + pix];
                if (corr) v = corr_apply(v, corr[pix_off + pix]);
            } else {
                v = x[pix_off + pix];
            }
        }
        xv[u] = v;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r0 = (rw[u] >> kBandShift) & 3;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = r - r0;
            if (j >= 0 && j < n[u]) {
                const T cv = j == 0 ? c[u][0] : j == 1 ? c[u][1] : j == 2 ? c[u][2] : c[u][3];
                a[r].add(cv, xv[u]);
            }
        }
    }
}

// Maps workgroup g of Gd onto its pieces: one per workgroup when Gd covers
// them, otherwise each XCD (g % 8) walks one contiguous eighth.
__device__ __forceinline__ void piece_range(int32_t g, int32_t Gd, int32_t npieces,
                                            int32_t& t_begin, int32_t& t_end,
                                            int32_t& t_step) {
    if (Gd < 8) {
        t_begin = g; t_end = npieces; t_step = Gd;
    } else {
        const int32_t xcd = g & 7, q = g >> 3, nq = (Gd - xcd + 7) >> 3;
        const int32_t per = npieces >> 3, rem = npieces & 7;
        const int32_t t0 = xcd * per + min(xcd, rem);
        t_begin = t0 + q; t_end = t0 + per + (xcd < rem ? 1 : 0); t_step = nq;
    }
}

// One workgroup per piece of one band: the wavefronts take the piece's
// groups in turn, U in flight each; the R row sums are reduced over the
// workgroup in a fixed tree and written to the piece's partial slots.
template <class T, class Acc, int U, int BLOCK, class RawT = T, bool kCorr = false,
          class CorrT = typename Pair2<T>::type>
__global__ __launch_bounds__(BLOCK) void k_band_runs(const BandPiece* __restrict__ pieces,
                                                   int32_t npieces,
                                                   const int32_t* __restrict__ runs,
                                                   const int32_t* __restrict__ gbase,
                                                   const T* __restrict__ coef,
                                                   const T* __restrict__ x,
                                                   Acc* __restrict__ parts,
                                                   const RawT* __restrict__ raw = nullptr,
                                                   const CorrT* __restrict__ corr = nullptr) {
    constexpr int R = kRunRows;
    __shared__ Acc red[BLOCK / kWave][R];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid & (kWave - 1);
    int32_t t_begin, t_end, t_step;
    piece_range(blockIdx.x, gridDim.x, npieces, t_begin, t_end, t_step);
    for (int32_t ti = t_begin; ti < t_end; ti += t_step) {
        const BandPiece pc = pieces[ti];
        Acc a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r].zero();
        for (int32_t z0 = pc.z0 + wave * kWave; z0 < pc.z1; z0 += BLOCK * U)
            run_groups<T, Acc, U, RawT, kCorr, CorrT>(z0, BLOCK, pc.z1, lane, runs, gbase, coef,
                                                      x, raw, corr, pc.pix_off, a);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            group_reduce(a[r], kWave);
            if (lane == 0) red[wave][r] = a[r];
        }
        __syncthreads();
        if (tid < R) {
            Acc sacc = red[0][tid];
            for (int k = 1; k < BLOCK / kWave; ++k) sacc.merge(red[k][tid]);
            parts[pc.slot0 + tid] = sacc;
        }
        __syncthreads();
    }
}

// Co-scheduled bands: a workgroup of WAVES wavefronts takes WAVES
// neighbouring bands over one stretch of image rows, wavefront w walking
// band w's runs of those rows (entry ti * WAVES + w of the schedule).
// Neighbouring bands are neighbouring rings, so the wavefronts of a
// workgroup gather from the same image lines at about the same time and
// share them in the CU's L1 cache.  Each wavefront reduces its own band's
// R row sums and writes them to its partial slots: no LDS, no barrier.
template <class T, class Acc, int U, int WAVES, class RawT = T, bool kCorr = false,
          class CorrT = typename Pair2<T>::type>
__global__ __launch_bounds__(WAVES * kWave) void k_runs_grouped(
    const BandPiece* __restrict__ pieces, int32_t ntiles, const int32_t* __restrict__ runs,
    const int32_t* __restrict__ gbase, const T* __restrict__ coef, const T* __restrict__ x,
    typename Acc::Slot* __restrict__ parts, const RawT* __restrict__ raw = nullptr,
    const CorrT* __restrict__ corr = nullptr) {
    constexpr int R = kRunRows;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    int32_t t_begin, t_end, t_step;
    piece_range(blockIdx.x, gridDim.x, ntiles, t_begin, t_end, t_step);
    for (int32_t ti = t_begin; ti < t_end; ti += t_step) {
        const BandPiece pc = pieces[(int64_t)ti * WAVES + wave];
        Acc a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r].zero();
        for (int32_t z0 = pc.z0; z0 < pc.z1; z0 += kWave * U)
            run_groups<T, Acc, U, RawT, kCorr, CorrT>(z0, kWave, pc.z1, lane, runs, gbase, coef,
                                                      x, raw, corr, pc.pix_off, a);
#pragma unroll
        for (int r = 0; r < R; ++r) group_reduce(a[r], kWave);
        if (lane == 0 && pc.slot0 >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) parts[pc.slot0 + r] = a[r].slot();
        }
    }
}

// One wavefront per bin adds the partial sums of its band's pieces (slots
// first, first + R, ...) in a fixed order and writes W, U and I.
template <class T, class Acc>
__global__ void k_band_reduce(const int32_t* __restrict__ bin_slot,
                              const int32_t* __restrict__ bin_count, int32_t R, int64_t b0,
                              int64_t b1, const Acc* __restrict__ parts, T* __restrict__ I,
                              T* __restrict__ W, T* __restrict__ U, double empty,
                              const double* __restrict__ ufix_in, double* __restrict__ ufix_out,
                              const double* __restrict__ wsub_in, double* __restrict__ wfix_out) {
    const int64_t b = b0 + (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (b >= b1) return;
    const int lane = threadIdx.x & (kWave - 1);
    Acc a;
    a.zero();
    const int32_t first = bin_slot[b], cnt = bin_count[b];
    const RowFixed f = load_row_fixed(b, ufix_in, wsub_in);
    for (int32_t k = lane; k < cnt; k += kWave) a.merge(parts[first + (int64_t)k * R]);
    group_reduce(a, kWave);
    if (lane == 0) write_row_u((int32_t)b, a, I, W, U, empty, f, ufix_out, wfix_out);
}

// One lane per bin, for matrices whose bins have at most kLaneParts
// partials.  The lane combines them as lane 0 of k_band_reduce's xor tree
// does (partial k with k + 4, then k + 2, then k + 1; the tree's wider steps
// only add zeros, which leave the sums unchanged), so both forms write the
// same bits.  It launches 64 times fewer wavefronts, which matters for
// batches of many small images, where most bins have one or two partials.
constexpr int kLaneParts = 8;

template <class T, class Acc>
__global__ void k_band_reduce_lane(const int32_t* __restrict__ bin_slot,
                                   const int32_t* __restrict__ bin_count, int32_t R, int64_t b0,
                                   int64_t b1, const Acc* __restrict__ parts, T* __restrict__ I,
                                   T* __restrict__ W, T* __restrict__ U, double empty,
                                   const double* __restrict__ ufix_in,
                                   double* __restrict__ ufix_out,
                                   const double* __restrict__ wsub_in,
                                   double* __restrict__ wfix_out) {
    const int64_t b = b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= b1) return;
    const int32_t first = bin_slot[b], cnt = bin_count[b];
    const RowFixed f = load_row_fixed(b, ufix_in, wsub_in);
    Acc v[kLaneParts];
#pragma unroll
    for (int k = 0; k < kLaneParts; ++k) {
        v[k].zero();
        if (k < cnt) v[k].merge(parts[first + (int64_t)k * R]);
    }
#pragma unroll
    for (int m = kLaneParts / 2; m > 0; m >>= 1) {
#pragma unroll
        for (int k = 0; k < m; ++k) v[k].merge(v[k + m]);
    }
    write_row_u((int32_t)b, v[0], I, W, U, empty, f, ufix_out, wfix_out);
}

// ---------------------------------------------------------------------------
// Blocked form: one workgroup per image tile
// ---------------------------------------------------------------------------

// Reads the tile's pixels row-major (coalesced), applies the cast and the
// correction map of Section 6.4 on the way (dark / norm may be null), keeps
// the corrected values in LDS, then sums every bin the tile feeds over its
// entries -- a small gather product from LDS -- into that (tile, bin)'s
// partial slot.  A group of G lanes takes one bin row at a time.
template <class R, class T, class Acc, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_block(const BlockTile* __restrict__ tiles,
                                                 int32_t ntiles,
                                                 const BlockRow* __restrict__ rows,
                                                 const uint16_t* __restrict__ lp,
                                                 const T* __restrict__ coef,
                                                 const R* __restrict__ img,
                                                 const T* __restrict__ dark,
                                                 const T* __restrict__ norm,
                                                 Acc* __restrict__ parts) {
    constexpr int U = 4;
    __shared__ T xs[kStageTileH * kStageTileW];
    const int tid = threadIdx.x;
    const int32_t g = blockIdx.x, Gd = gridDim.x;
    // XCD-contiguous ranges of tiles, as in k_spmv
    int32_t t_begin, t_end, t_step;
    if (Gd < 8) {
        t_begin = g; t_end = ntiles; t_step = Gd;
    } else {
        const int32_t xcd = g & 7, q = g >> 3, nq = (Gd - xcd + 7) >> 3;
        const int32_t per = ntiles >> 3, rem = ntiles & 7;
        const int32_t t0 = xcd * per + min(xcd, rem);
        t_begin = t0 + q; t_end = t0 + per + (xcd < rem ? 1 : 0); t_step = nq;
    }
    for (int32_t ti = t_begin; ti < t_end; ti += t_step) {
        const BlockTile t = tiles[ti];
        const int32_t n = t.th * t.tw;
        for (int32_t e = tid; e < n; e += BLOCK) {
            const int32_t r = e / t.tw, c = e - r * t.tw;
            const int64_t p = t.img_off + (int64_t)(t.i0 + r) * t.w + t.j0 + c;
            T v = (T)img[p];
            if (dark) v = v - dark[p];
            if (norm) v = v / norm[p];
            xs[e] = v;
        }
        __syncthreads();
        const BlockRow* tr = rows + t.row_off;
        const uint16_t* tl = lp + t.ent_off;
        const T* tc = coef + t.ent_off;
        const int32_t nr = t.nrows;
        const int32_t nent = nr > 0 ? tr[nr - 1].end : 0;
        const int32_t avg = nr > 0 ? (nent + nr - 1) / nr : 0;
        int G = 1;
        while (G < kWave && 2 * G < avg) G <<= 1;
        while (G < kWave && nr * G < BLOCK) G <<= 1;
        const int ngroups = BLOCK / G;
        const int grp = tid / G, lane = tid & (G - 1);
        for (int32_t r = grp; r < nr; r += ngroups) {
            const BlockRow row = tr[r];
            Acc a;
            a.zero();
            for (int32_t k = row.start + lane; k < row.end; k += G * U) {
                uint16_t li[U];
                T cv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t kk = k + u * G;
                    if (kk < row.end) {
                        li[u] = tl[kk];
                        cv[u] = tc[kk];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (k + u * G < row.end) a.add(cv[u], xs[li[u]]);
            }
            group_reduce(a, G);
            if (lane == 0) parts[row.slot] = a;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// Correction map (Section 6.4)
// ---------------------------------------------------------------------------


// x[i] = (T(raw[src]) - dark[i]) / norm[i], src = order ? order[i] : i.
// With a ring order the output is the image in ring positions (and dark and
// norm are given in that order too); without one it is row-major.
template <class R, class T>
__global__ void k_correct(const R* __restrict__ raw, const int32_t* __restrict__ order,
                          const T* __restrict__ dark, const T* __restrict__ norm,
                          T* __restrict__ x, int64_t n) {
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i0 = b * (int64_t)blockDim.x * 4 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + (int64_t)k * blockDim.x;
        if (i < n) {
            T v = (T)raw[order ? (int64_t)order[i] : i];
            if (dark) v = v - dark[i];
            if (norm) v = v / norm[i];
            x[i] = v;
        }
    }
}

// Ring staging, scatter form: pixels [p0, p1) are read row-major (coalesced)
// and written to their ring positions x[pos[p]].
template <class R, class T>
__global__ void k_stage_scatter(const R* __restrict__ raw, const int32_t* __restrict__ pos,
                                const T* __restrict__ dark, const T* __restrict__ norm,
                                T* __restrict__ x, int64_t p0, int64_t p1) {
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i0 = p0 + b * (int64_t)blockDim.x * 4 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t p = i0 + (int64_t)k * blockDim.x;
        if (p < p1) {
            T v = (T)raw[p];
            if (dark) v = v - dark[p];
            if (norm) v = v / norm[p];
            x[pos[p]] = v;
        }
    }
}

// Ring staging through LDS: one workgroup per image tile reads the tile's
// pixels row-major (coalesced), drops each corrected value at its rank among
// the tile's ring positions, then writes the ranks out in order -- runs of
// consecutive ring positions, so the stores are contiguous too.
template <class R, class T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_stage_tile(const StageTile* __restrict__ tiles,
                                                      const R* __restrict__ raw,
                                                      const uint16_t* __restrict__ lidx,
                                                      const int32_t* __restrict__ dest,
                                                      const T* __restrict__ dark,
                                                      const T* __restrict__ norm,
                                                      T* __restrict__ x) {
    __shared__ T buf[kStageTileH * kStageTileW];
    const StageTile st = tiles[xcd_block(blockIdx.x, gridDim.x)];
    const int32_t n = st.th * st.tw;
    for (int32_t e = threadIdx.x; e < n; e += BLOCK) {
        const int32_t r = e / st.tw, c = e - r * st.tw;
        const int64_t p = st.img_off + (int64_t)(st.i0 + r) * st.w + st.j0 + c;
        T v = (T)raw[p];
        if (dark) v = v - dark[p];
        if (norm) v = v / norm[p];
        buf[lidx[st.k_off + e]] = v;
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < n; k += BLOCK) x[dest[st.k_off + k]] = buf[k];
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

// One thread per pixel over its pixel-major entries, ascending bins.  A
// pixel has a handful of entries (2.8 on average with bounding-box
// splitting); the first four are loaded before any is used, so a lane keeps
// its loads in flight instead of waiting entry by entry.  Consecutive lanes
// read consecutive stretches of the entry arrays.  With kFirst the bins of
// a pixel are consecutive and given by the pixel's first bin alone (one
// word per pixel instead of one per entry).
// Four consecutive values from a 4-byte (float) or 8-byte (double)
// aligned address, as one or two vector loads.
typedef float F4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double D2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ inline void load4u(const float* p, float v[4]) {
    const F4u a = *reinterpret_cast<const F4u*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ inline void load4u(const double* p, double v[4]) {
    const D2u a = *reinterpret_cast<const D2u*>(p);
    const D2u b = *reinterpret_cast<const D2u*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <class T, bool kFirst>
__global__ void k_csc_bwd(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                          const int32_t* __restrict__ first, const T* __restrict__ cdata,
                          const double* __restrict__ v, const T* __restrict__ norm,
                          T* __restrict__ gx, int64_t npix) {
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int32_t k0 = colptr[p], k1 = colptr[p + 1];
    T c[4];
    double vb[4];
    int32_t b0 = 0;
    if constexpr (kFirst) {
        // the pixel's first four coefficients and the values of its first
        // four bins (consecutive) in two vector loads each; entries past
        // the pixel's count are read (the arrays keep spare elements) and
        // not used
        b0 = first[p];
        load4u(cdata + k0, c);
        load4u(v + b0, vb);
    } else {
        int32_t b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (k0 + j < k1) {
                c[j] = cdata[k0 + j];
                b[j] = rowidx[k0 + j];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) vb[j] = (k0 + j < k1) ? v[b[j]] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (k0 + j < k1) acc = __fma_rn((double)c[j], vb[j], acc);
    for (int32_t k = k0 + 4; k < k1; ++k)
        acc = __fma_rn((double)cdata[k], v[kFirst ? b0 + (k - k0) : rowidx[k]], acc);
    if (norm) acc = acc / (double)norm[p];
    gx[p] = (T)acc;
}

int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

template <class T, class Acc, int BLOCK, int VAR>
hipError_t forward_impl(const ForwardLaunch& a, hipStream_t s) {
    if (a.ntiles > 0) {
        const int grid = a.grid > 0 ? a.grid : a.ntiles;
        hipLaunchKernelGGL((k_spmv<T, Acc, BLOCK, VAR>), dim3(grid), dim3(BLOCK), 0, s,
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

template <class T, class Acc, int VAR>
hipError_t forward_var(const ForwardLaunch& a, hipStream_t s) {
    switch (a.block) {
        case 64: return forward_impl<T, Acc, 64, VAR>(a, s);
        case 128: return forward_impl<T, Acc, 128, VAR>(a, s);
        case 256: return forward_impl<T, Acc, 256, VAR>(a, s);
        case 512: return forward_impl<T, Acc, 512, VAR>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, class Acc>
hipError_t forward_block(const ForwardLaunch& a, hipStream_t s) {
    static_assert(kVariants == kNumVariants, "variant table");
    switch (a.variant) {
        case 0: return forward_var<T, Acc, 0>(a, s);
        case 1: return forward_var<T, Acc, 1>(a, s);
        case 2: return forward_var<T, Acc, 2>(a, s);
        case 3: return forward_var<T, Acc, 3>(a, s);
        case 4: return forward_var<T, Acc, 4>(a, s);
        case 5: return forward_var<T, Acc, 5>(a, s);
        case 6: return forward_var<T, Acc, 6>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class R, class T>
hipError_t correct_impl(const void* raw, const int32_t* order, const void* dark, const void* norm,
                        void* x, int64_t n, hipStream_t s) {
    const int64_t blocks = (n + 1023) / 1024;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_correct<R, T>), dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const R*>(raw), order, static_cast<const T*>(dark),
                       static_cast<const T*>(norm), static_cast<T*>(x), n);
    return hipGetLastError();
}

template <class T>
hipError_t correct_raw(const void* raw, int32_t raw_dtype, const int32_t* order, const void* dark,
                       const void* norm, void* x, int64_t n, hipStream_t s) {
    switch (raw_dtype) {
        case AZI_I16: return correct_impl<int16_t, T>(raw, order, dark, norm, x, n, s);
        case AZI_U16: return correct_impl<uint16_t, T>(raw, order, dark, norm, x, n, s);
        case AZI_I32: return correct_impl<int32_t, T>(raw, order, dark, norm, x, n, s);
        case AZI_U32: return correct_impl<uint32_t, T>(raw, order, dark, norm, x, n, s);
        case AZI_F32: return correct_impl<float, T>(raw, order, dark, norm, x, n, s);
        case AZI_F64: return correct_impl<double, T>(raw, order, dark, norm, x, n, s);
        default: return hipErrorInvalidValue;
    }
}

template <class R, class T>
hipError_t stage_impl(const StageLaunch& a, hipStream_t s) {
    const R* raw = static_cast<const R*>(a.raw);
    const T* dark = static_cast<const T*>(a.dark);
    const T* norm = static_cast<const T*>(a.norm);
    T* x = static_cast<T*>(a.x);
    if (a.mode == kStageScatter) {
        const int64_t n = a.p1 - a.p0;
        if (n <= 0) return hipSuccess;
        const int64_t blocks = (n + 1023) / 1024;
        hipLaunchKernelGGL((k_stage_scatter<R, T>), dim3((unsigned)blocks), dim3(256), 0, s, raw,
                           a.pos, dark, norm, x, a.p0, a.p1);
    } else {
        if (a.ntiles <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_stage_tile<R, T, 256>), dim3((unsigned)a.ntiles), dim3(256), 0, s,
                           a.tiles, raw, a.lidx, a.dest, dark, norm, x);
    }
    return hipGetLastError();
}

template <class T>
hipError_t stage_raw(const StageLaunch& a, hipStream_t s) {
    switch (a.raw_dtype) {
        case AZI_I16: return stage_impl<int16_t, T>(a, s);
        case AZI_U16: return stage_impl<uint16_t, T>(a, s);
        case AZI_I32: return stage_impl<int32_t, T>(a, s);
        case AZI_U32: return stage_impl<uint32_t, T>(a, s);
        case AZI_F32: return stage_impl<float, T>(a, s);
        case AZI_F64: return stage_impl<double, T>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, class Acc, int BLOCK, int R>
hipError_t band_launch(const BandLaunch& a, hipStream_t s) {
    const int grid = a.grid > 0 ? a.grid : a.npieces;
    hipLaunchKernelGGL((k_band<T, Acc, BLOCK, R>), dim3(grid), dim3(BLOCK), 0, s, a.pieces,
                       a.npieces, a.packed, static_cast<const T*>(a.coef),
                       static_cast<const T*>(a.x), static_cast<Acc*>(a.parts),
                       static_cast<const T*>(nullptr),
                       static_cast<const typename Pair2<T>::type*>(nullptr));
    return hipGetLastError();
}

// Raw-frame form (256 threads): cast and correction in the gather.
template <class T, class Acc, int R, class RawT>
hipError_t band_launch_raw(const BandLaunch& a, hipStream_t s) {
    const int grid = a.grid > 0 ? a.grid : a.npieces;
    if constexpr (std::is_same<T, double>::value) {
        if (a.corr && a.corr_kind == kCorrRecord12) {
            hipLaunchKernelGGL((k_band<T, Acc, 256, R, RawT, true, Corr12>), dim3(grid), dim3(256),
                               0, s, a.pieces, a.npieces, a.packed, static_cast<const T*>(a.coef),
                               static_cast<const T*>(nullptr), static_cast<Acc*>(a.parts),
                               static_cast<const RawT*>(a.raw), static_cast<const Corr12*>(a.corr));
            return hipGetLastError();
        }
    }
    if (a.corr_kind != kCorrPair) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_band<T, Acc, 256, R, RawT, true>), dim3(grid), dim3(256), 0, s,
                       a.pieces, a.npieces, a.packed, static_cast<const T*>(a.coef),
                       static_cast<const T*>(nullptr), static_cast<Acc*>(a.parts),
                       static_cast<const RawT*>(a.raw),
                       static_cast<const typename Pair2<T>::type*>(a.corr));
    return hipGetLastError();
}

template <class T, class Acc, int R>
hipError_t band_raw(const BandLaunch& a, hipStream_t s) {
    switch (a.raw_dtype) {
        case AZI_I16: return band_launch_raw<T, Acc, R, int16_t>(a, s);
        case AZI_U16: return band_launch_raw<T, Acc, R, uint16_t>(a, s);
        case AZI_I32: return band_launch_raw<T, Acc, R, int32_t>(a, s);
        case AZI_U32: return band_launch_raw<T, Acc, R, uint32_t>(a, s);
        case AZI_F32: return band_launch_raw<T, Acc, R, float>(a, s);
        case AZI_F64: return band_launch_raw<T, Acc, R, double>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, class Acc, int R>
hipError_t band_block(const BandLaunch& a, hipStream_t s) {
    if (a.raw) return band_raw<T, Acc, R>(a, s);
    switch (a.block) {
        case 64:
        case 128: return band_launch<T, Acc, 128, R>(a, s);
        case 256: return band_launch<T, Acc, 256, R>(a, s);
        case 512: return band_launch<T, Acc, 512, R>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Groups in flight per wavefront (measured at 1e7 pixels: 2 for float64,
// 4 for float32, whose registers are half the size; one more when the
// accumulator holds W alone, which frees the registers of another group
// within the 64 VGPRs of 8 wavefronts per SIMD: float64 60, float32 62 at
// most over the raw types and dark forms).
template <class T, class Acc>
constexpr int kRunGroups = std::is_same<Acc, AccWF64>::value ? (sizeof(T) == 8 ? 3 : 5)
                                                            : (sizeof(T) == 8 ? 2 : 4);

// The co-scheduled kernel of `a.waves` bands per workgroup, accumulating in
// Acc (partial-sum slots of Acc::Slot).
template <class T, class Acc, class RawT, bool kCorr, class CorrT>
hipError_t grouped_launch(const BandLaunch& a, const T* x, hipStream_t s) {
    constexpr int G = kRunGroups<T, Acc>;
    const T* coef = static_cast<const T*>(a.coef);
    auto* parts = static_cast<typename Acc::Slot*>(a.parts);
    const RawT* raw = static_cast<const RawT*>(a.raw);
    const CorrT* corr = static_cast<const CorrT*>(a.corr);
    const int32_t ntiles = a.npieces / a.waves;
    const int grid = a.grid > 0 ? a.grid : ntiles;
    if (ntiles <= 0) return hipSuccess;
    if (a.waves == 4)
        hipLaunchKernelGGL((k_runs_grouped<T, Acc, G, 4, RawT, kCorr, CorrT>), dim3(grid),
                           dim3(4 * kWave), 0, s, a.pieces, ntiles, a.packed, a.gbase, coef, x,
                           parts, raw, corr);
    else if (a.waves == 8)
        hipLaunchKernelGGL((k_runs_grouped<T, Acc, G, 8, RawT, kCorr, CorrT>), dim3(grid),
                           dim3(8 * kWave), 0, s, a.pieces, ntiles, a.packed, a.gbase, coef, x,
                           parts, raw, corr);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Launches the run-layout kernel of the launch's form: one band per
// workgroup of a.block threads (a.waves == 1), or a.waves co-scheduled
// bands per workgroup.  A raw-frame launch that takes U from the plan
// (ufix_in: the folded coefficients) accumulates W alone.
template <class T, class Acc, class RawT, bool kCorr, class CorrT>
hipError_t runs_kernel(const BandLaunch& a, const T* x, hipStream_t s) {
    constexpr int G = kRunGroups<T, Acc>;
    const T* coef = static_cast<const T*>(a.coef);
    Acc* parts = static_cast<Acc*>(a.parts);
    const RawT* raw = static_cast<const RawT*>(a.raw);
    const CorrT* corr = static_cast<const CorrT*>(a.corr);
    if (a.waves > 1) {
        if constexpr (kCorr && IsRunDark<CorrT>::value) {
            // a dark value per run exists only with the folded coefficients,
            // whose U is the plan's
            if (!a.ufix_in) return hipErrorInvalidValue;
            return grouped_launch<T, typename WOnly<Acc>::type, RawT, kCorr, CorrT>(a, x, s);
        } else {
            if (kCorr && a.ufix_in)
                return grouped_launch<T, typename WOnly<Acc>::type, RawT, kCorr, CorrT>(a, x, s);
            return grouped_launch<T, Acc, RawT, kCorr, CorrT>(a, x, s);
        }
    }
    const int grid = a.grid > 0 ? a.grid : a.npieces;
    if (a.block == 128)
        hipLaunchKernelGGL((k_band_runs<T, Acc, G, 128, RawT, kCorr, CorrT>), dim3(grid),
                           dim3(128), 0, s, a.pieces, a.npieces, a.packed, a.gbase, coef, x, parts,
                           raw, corr);
    else
        hipLaunchKernelGGL((k_band_runs<T, Acc, G, 256, RawT, kCorr, CorrT>), dim3(grid),
                           dim3(256), 0, s, a.pieces, a.npieces, a.packed, a.gbase, coef, x, parts,
                           raw, corr);
    return hipGetLastError();
}

template <class T, class Acc0, int WAVES>
int32_t runs_resident() {
    using Acc = typename WOnly<Acc0>::type;  // the folded raw-frame form
    int n = 0;
    const void* f = reinterpret_cast<const void*>(
        &k_runs_grouped<T, Acc, kRunGroups<T, Acc>, WAVES, int32_t, true, RunDark<float>>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, WAVES * kWave, 0) != hipSuccess)
        return 0;
    return n;
}

template <class T, class Acc, class RawT, class CorrT>
hipError_t runs_launch_raw(const BandLaunch& a, int, hipStream_t s) {
    return runs_kernel<T, Acc, RawT, true, CorrT>(a, nullptr, s);
}

template <class T, class Acc, class RawT>
hipError_t runs_raw_corr(const BandLaunch& a, int grid, hipStream_t s) {
    if constexpr (std::is_same<T, double>::value) {
        if (a.corr && a.corr_kind == kCorrRecord12)
            return runs_launch_raw<T, Acc, RawT, Corr12>(a, grid, s);
        if (a.corr && a.corr_kind == kCorrRunDarkF32)
            return runs_launch_raw<T, Acc, RawT, RunDark<float>>(a, grid, s);
    }
    if (a.corr && a.corr_kind == kCorrRunDark)
        return runs_launch_raw<T, Acc, RawT, RunDark<T>>(a, grid, s);
    if (a.corr && a.corr_kind == kCorrRunDarkU16)
        return runs_launch_raw<T, Acc, RawT, RunDark<uint16_t>>(a, grid, s);
    if (a.corr_kind != kCorrPair && a.corr) return hipErrorInvalidValue;
    return runs_launch_raw<T, Acc, RawT, typename Pair2<T>::type>(a, grid, s);
}

template <class T, class Acc>
hipError_t runs_launch(const BandLaunch& a, hipStream_t s) {
    const int grid = a.grid > 0 ? a.grid : a.npieces;
    if (!a.raw)
        return runs_kernel<T, Acc, T, false, typename Pair2<T>::type>(
            a, static_cast<const T*>(a.x), s);
    switch (a.raw_dtype) {
        case AZI_I16: return runs_raw_corr<T, Acc, int16_t>(a, grid, s);
        case AZI_U16: return runs_raw_corr<T, Acc, uint16_t>(a, grid, s);
        case AZI_I32: return runs_raw_corr<T, Acc, int32_t>(a, grid, s);
        case AZI_U32: return runs_raw_corr<T, Acc, uint32_t>(a, grid, s);
        case AZI_F32: return runs_raw_corr<T, Acc, float>(a, grid, s);
        case AZI_F64: return runs_raw_corr<T, Acc, double>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, class Acc>
hipError_t band_impl(const BandLaunch& a, hipStream_t s) {
    if (a.npieces > 0 && a.gbase) {
        if (a.R != kRunRows) return hipErrorInvalidValue;
        const hipError_t e = runs_launch<T, Acc>(a, s);
        if (e != hipSuccess) return e;
    } else if (a.npieces > 0) {
        hipError_t e;
        switch (a.R) {
            case 4: e = band_block<T, Acc, 4>(a, s); break;
            case 8: e = band_block<T, Acc, 8>(a, s); break;
            case 16: e = band_block<T, Acc, 16>(a, s); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    const int64_t nb = a.b1 - a.b0;
    if (nb > 0 && a.max_count <= kLaneParts) {
        hipLaunchKernelGGL((k_band_reduce_lane<T, Acc>), dim3((unsigned)((nb + 255) / 256)),
                           dim3(256), 0, s, a.bin_slot, a.bin_count, a.R, a.b0, a.b1,
                           static_cast<const Acc*>(a.parts), static_cast<T*>(a.I),
                           static_cast<T*>(a.W), static_cast<T*>(a.U), a.empty, a.ufix_in,
                           a.ufix_out, a.wsub_in, a.wfix_out);
        return hipGetLastError();
    }
    if (nb > 0) {
        hipLaunchKernelGGL((k_band_reduce<T, Acc>), dim3((unsigned)((nb + 3) / 4)), dim3(256), 0,
                           s, a.bin_slot, a.bin_count, a.R, a.b0, a.b1,
                           static_cast<const Acc*>(a.parts), static_cast<T*>(a.I),
                           static_cast<T*>(a.W), static_cast<T*>(a.U), a.empty, a.ufix_in,
                           a.ufix_out, a.wsub_in, a.wfix_out);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <class R, class T, class Acc>
hipError_t block_impl(const BlockLaunch& a, hipStream_t s) {
    if (a.ntiles > 0) {
        const int grid = a.grid > 0 ? a.grid : a.ntiles;
        const R* img = static_cast<const R*>(a.img);
        const T* dark = static_cast<const T*>(a.dark);
        const T* norm = static_cast<const T*>(a.norm);
        const T* coef = static_cast<const T*>(a.coef);
        Acc* parts = static_cast<Acc*>(a.parts);
        switch (a.block) {
            case 64:   // a tile needs more than one wavefront: smallest is 128
            case 128:
                hipLaunchKernelGGL((k_block<R, T, Acc, 128>), dim3(grid), dim3(128), 0, s, a.tiles,
                                   a.ntiles, a.rows, a.lp, coef, img, dark, norm, parts);
                break;
            case 256:
                hipLaunchKernelGGL((k_block<R, T, Acc, 256>), dim3(grid), dim3(256), 0, s, a.tiles,
                                   a.ntiles, a.rows, a.lp, coef, img, dark, norm, parts);
                break;
            case 512:
                hipLaunchKernelGGL((k_block<R, T, Acc, 512>), dim3(grid), dim3(512), 0, s, a.tiles,
                                   a.ntiles, a.rows, a.lp, coef, img, dark, norm, parts);
                break;
            default:
                return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t nb = a.b1 - a.b0;
    if (nb > 0) {
        const int64_t blocks = (nb + 3) / 4;
        hipLaunchKernelGGL((k_block_reduce<T, Acc>), dim3((unsigned)blocks), dim3(256), 0, s,
                           a.bin_ptr, a.b0, a.b1, static_cast<const Acc*>(a.parts),
                           static_cast<T*>(a.I), static_cast<T*>(a.W), static_cast<T*>(a.U),
                           a.empty);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <class T, class Acc>
hipError_t block_raw(const BlockLaunch& a, hipStream_t s) {
    switch (a.img_dtype) {
        case AZI_I16: return block_impl<int16_t, T, Acc>(a, s);
        case AZI_U16: return block_impl<uint16_t, T, Acc>(a, s);
        case AZI_I32: return block_impl<int32_t, T, Acc>(a, s);
        case AZI_U32: return block_impl<uint32_t, T, Acc>(a, s);
        case AZI_F32: return block_impl<float, T, Acc>(a, s);
        case AZI_F64: return block_impl<double, T, Acc>(a, s);
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
        const int64_t blocks = (a.npix + 255) / 256;
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        if (a.first)
            hipLaunchKernelGGL((k_csc_bwd<T, true>), dim3((unsigned)blocks), dim3(256), 0, s,
                               a.colptr, a.rowidx, a.first, static_cast<const T*>(a.cdata), a.v,
                               static_cast<const T*>(a.norm), static_cast<T*>(a.gx), a.npix);
        else
            hipLaunchKernelGGL((k_csc_bwd<T, false>), dim3((unsigned)blocks), dim3(256), 0, s,
                               a.colptr, a.rowidx, a.first, static_cast<const T*>(a.cdata), a.v,
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

hipError_t launch_correct(const void* raw, int32_t raw_dtype, const int32_t* order,
                          const void* dark, const void* norm, void* x, int32_t dtype, int64_t n,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return dtype == AZI_F64 ? correct_raw<double>(raw, raw_dtype, order, dark, norm, x, n, s)
                            : correct_raw<float>(raw, raw_dtype, order, dark, norm, x, n, s);
}

namespace {
// pair[i] = (dark[i] or 0, 1 / norm[i] or 1): the fused gather's correction.
template <class T>
__global__ void k_corr_pair(const T* __restrict__ dark, const T* __restrict__ norm,
                            typename Pair2<T>::type* __restrict__ pair, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename Pair2<T>::type v;
    v.x = dark ? dark[i] : T(0);
    v.y = norm ? T(1) / norm[i] : T(1);
    pair[i] = v;
}
}  // namespace

namespace {
// flag[0] = 1 when some dark[i] does not survive the round trip through
// float (every writer stores the same 1, so their order does not matter).
__global__ void k_dark_is_float(const double* __restrict__ dark, int64_t n,
                                int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = dark[i];
    if (!((double)(float)d == d)) flag[0] = 1;
}

__global__ void k_corr_record12(const double* __restrict__ dark, const double* __restrict__ norm,
                                Corr12* __restrict__ rec, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = norm ? 1.0 / norm[i] : 1.0;
    Corr12 r;
    r.dark = (float)dark[i];
    r.inv_lo = (uint32_t)__double2loint(inv);
    r.inv_hi = (uint32_t)__double2hiint(inv);
    rec[i] = r;
}
}  // namespace

hipError_t launch_dark_is_float(const double* dark, int64_t n, int32_t* flag, hipStream_t s) {
    hipError_t e = hipMemsetAsync(flag, 0, 4, s);
    if (e != hipSuccess || n <= 0) return e;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dark_is_float, dim3((unsigned)blocks), dim3(256), 0, s, dark, n, flag);
    return hipGetLastError();
}

hipError_t launch_corr_record12(const double* dark, const double* norm, void* rec, int64_t n,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_corr_record12, dim3((unsigned)blocks), dim3(256), 0, s, dark, norm,
                       static_cast<Corr12*>(rec), n);
    return hipGetLastError();
}

hipError_t launch_corr_pair(const void* dark, const void* norm, void* pair, int32_t dtype,
                            int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (dtype == AZI_F64)
        hipLaunchKernelGGL(k_corr_pair<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const double*>(dark), static_cast<const double*>(norm),
                           static_cast<double2*>(pair), n);
    else
        hipLaunchKernelGGL(k_corr_pair<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const float*>(dark), static_cast<const float*>(norm),
                           static_cast<float2*>(pair), n);
    return hipGetLastError();
}

int32_t runs_resident_per_cu(int32_t dtype, int32_t accum, int32_t waves) {
    const bool k32 = dtype == AZI_F32 && accum == AZI_ACC_KAHAN32;
    if (waves == 4)
        return dtype == AZI_F64 ? runs_resident<double, AccF64, 4>()
               : k32            ? runs_resident<float, AccK32, 4>()
                                : runs_resident<float, AccF64, 4>();
    if (waves == 8)
        return dtype == AZI_F64 ? runs_resident<double, AccF64, 8>()
               : k32            ? runs_resident<float, AccK32, 8>()
                                : runs_resident<float, AccF64, 8>();
    return 0;
}

hipError_t launch_band(const BandLaunch& a, hipStream_t s) {
    if (a.dtype == AZI_F64) return band_impl<double, AccF64>(a, s);
    if (a.accum == AZI_ACC_KAHAN32) return band_impl<float, AccK32>(a, s);
    return band_impl<float, AccF64>(a, s);
}

hipError_t launch_block(const BlockLaunch& a, hipStream_t s) {
    if (a.dtype == AZI_F64) return block_raw<double, AccF64>(a, s);
    if (a.accum == AZI_ACC_KAHAN32) return block_raw<float, AccK32>(a, s);
    return block_raw<float, AccF64>(a, s);
}

hipError_t launch_stage(const StageLaunch& a, hipStream_t s) {
    if (a.mode == kStageGather)
        return launch_correct(a.raw, a.raw_dtype, a.order, a.dark, a.norm, a.x, a.dtype, a.p1 - a.p0,
                              s);
    return a.dtype == AZI_F64 ? stage_raw<double>(a, s) : stage_raw<float>(a, s);
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
