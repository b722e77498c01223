// Host plan builder: detector geometry -> per-pixel radial extent ->
// bounding-box coefficients (Section 4.1) or whole-pixel histogram entries
// (Section 3.3) -> pixel-major (CSC) and bin-major (CSR, Section 5.2.1)
// matrices -> tile schedule for the gather kernels.
//
// Compiled without floating-point contraction: every quantity that decides
// a bin index is formed by the same sequence of correctly rounded IEEE
// operations (+, -, *, /, sqrt, floor, ceil) as the plain definition, so
// the integer structure of the matrix is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <limits>

#include "internal.h"

namespace azi {
namespace {

// Output coordinate of a radius r in metres (Section 3 coordinate list):
// 2theta = atan(r / d), q = 4 pi sin(2theta / 2) / lambda with lambda in nm.
inline double to_unit(double r, int32_t unit, double dist, double wl) {
    switch (unit) {
        case AZI_UNIT_R_M: return r;
        case AZI_UNIT_R_MM: return r * 1e3;
        default: break;
    }
    const double tth = std::atan(r / dist);
    if (unit == AZI_UNIT_2TH_RAD) return tth;
    if (unit == AZI_UNIT_2TH_DEG) return tth * (180.0 / M_PI);
    return (4.0 * M_PI) * std::sin(tth / 2.0) / (wl * 1e9);
}

// Radial extent of pixel (i, j) = the square [j, j+1] x [i, i+1]: the
// farthest corner and the nearest point of the square from the beam centre
// (the box circumscribing the pixel in the radial direction), and the
// radius of the pixel midpoint.
struct Extent { double lo, hi, mid; };

inline Extent pixel_extent(int64_t i, int64_t j, const azi_geom& g) {
    const double cx = g.center_x_px, cy = g.center_y_px;
    const double px = g.pixel_x_m, py = g.pixel_y_m;
    const double x0 = ((double)j - cx) * px, x1 = ((double)(j + 1) - cx) * px;
    const double y0 = ((double)i - cy) * py, y1 = ((double)(i + 1) - cy) * py;
    const double a = x0 * x0, b = x1 * x1, c = y0 * y0, d = y1 * y1;
    const double s = std::max(std::max(a + c, b + c), std::max(a + d, b + d));
    const double ex = std::max(std::max((double)j - cx, cx - (double)(j + 1)), 0.0) * px;
    const double ey = std::max(std::max((double)i - cy, cy - (double)(i + 1)), 0.0) * py;
    const double xm = ((double)j + 0.5 - cx) * px, ym = ((double)i + 0.5 - cy) * py;
    Extent e;
    e.hi = std::sqrt(s);
    e.lo = std::sqrt(ex * ex + ey * ey);
    e.mid = std::sqrt(xm * xm + ym * ym);
    return e;
}

// Entries of one pixel for a box [lo, hi] over bins of width delta from
// pmin: fractional positions fl, fh; the inside part [flc, fhc] of [0, npt];
// bins floor(flc) .. ceil(fhc) - 1; weight = overlap / (fh - fl).
template <class Emit>
inline void bbox_pixel(double lo, double hi, double pmin, double delta, int32_t npt,
                       Emit&& emit) {
    const double fl = (lo - pmin) / delta;
    const double fh = (hi - pmin) / delta;
    const double n = (double)npt;
    if (fh == fl) {  // zero-width box: whole weight to its bin
        if (fl >= 0.0 && fl <= n) emit(std::min((int32_t)std::floor(fl), npt - 1), 1.0);
        return;
    }
    const double flc = std::max(fl, 0.0);
    const double fhc = std::min(fh, n);
    if (!(fhc > flc)) return;
    const double width = fh - fl;
    const int32_t b0 = (int32_t)std::floor(flc);
    const int32_t b1 = (int32_t)std::ceil(fhc) - 1;
    if (b0 == b1) {
        emit(b0, (fhc - flc) / width);
        return;
    }
    emit(b0, ((double)(b0 + 1) - flc) / width);
    const double inner = 1.0 / width;
    for (int32_t b = b0 + 1; b < b1; ++b) emit(b, inner);
    emit(b1, (fhc - (double)b1) / width);
}

}  // namespace

int build_matrix(const azi_geom& g, int32_t npt, int32_t unit, int32_t split,
                 const double* range2, HostMatrix& m, std::string& err) {
    const int64_t h = g.h, w = g.w, npix = h * w;
    if (npix >= (int64_t)std::numeric_limits<int32_t>::max()) {
        err = "image has 2^31 pixels or more";
        return AZI_EOVERFLOW;
    }
    std::vector<double> lo, hi;
    if (split == AZI_SPLIT_BBOX) { lo.resize(npix); hi.resize(npix); }
    else { lo.resize(npix); }  // pixel-midpoint values
    double mn = std::numeric_limits<double>::infinity(), mx = -mn;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < w; ++j) {
            const int64_t p = i * w + j;
            const Extent e = pixel_extent(i, j, g);
            if (split == AZI_SPLIT_BBOX) {
                lo[p] = to_unit(e.lo, unit, g.dist_m, g.wavelength_m);
                hi[p] = to_unit(e.hi, unit, g.dist_m, g.wavelength_m);
                mn = std::min(mn, lo[p]);
                mx = std::max(mx, hi[p]);
            } else {
                lo[p] = to_unit(e.mid, unit, g.dist_m, g.wavelength_m);
                mn = std::min(mn, lo[p]);
                mx = std::max(mx, lo[p]);
            }
        }
    }
    const double pmin = range2 ? range2[0] : mn;
    const double pmax = range2 ? range2[1] : mx;
    if (!(pmax > pmin) || !std::isfinite(pmin) || !std::isfinite(pmax)) {
        err = "integration range is empty or not finite";
        return AZI_EINVAL;
    }
    const double delta = (pmax - pmin) / npt;
    m.npt = npt;
    m.npix = npix;
    m.pmin = pmin;
    m.pmax = pmax;

    // Pixel-major pass: the CSC comes out in pixel order directly.
    m.colptr.assign(npix + 1, 0);
    m.rowidx.clear();
    m.cdata.clear();
    m.rowidx.reserve(split == AZI_SPLIT_BBOX ? npix * 3 : npix);
    m.cdata.reserve(m.rowidx.capacity());
    const int64_t limit = std::numeric_limits<int32_t>::max();
    for (int64_t p = 0; p < npix; ++p) {
        if (split == AZI_SPLIT_BBOX) {
            bbox_pixel(lo[p], hi[p], pmin, delta, npt, [&](int32_t b, double c) {
                m.rowidx.push_back(b);
                m.cdata.push_back(c);
            });
        } else {
            const double fc = (lo[p] - pmin) / delta;
            if (fc >= 0.0 && fc <= (double)npt) {
                m.rowidx.push_back(std::min((int32_t)std::floor(fc), npt - 1));
                m.cdata.push_back(1.0);
            }
        }
        if ((int64_t)m.rowidx.size() >= limit) {
            err = "matrix has 2^31 nonzeros or more";
            return AZI_EOVERFLOW;
        }
        m.colptr[p + 1] = (int32_t)m.rowidx.size();
    }

    // Transpose to CSR by counting sort; visiting pixels in ascending order
    // keeps every row's pixel ids ascending.
    const int64_t nnz = (int64_t)m.rowidx.size();
    m.indptr.assign(npt + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) m.indptr[m.rowidx[k] + 1]++;
    for (int32_t b = 0; b < npt; ++b) m.indptr[b + 1] += m.indptr[b];
    m.indices.resize(nnz);
    m.data.resize(nnz);
    std::vector<int32_t> cursor(m.indptr.begin(), m.indptr.end() - 1);
    for (int64_t p = 0; p < npix; ++p) {
        for (int32_t k = m.colptr[p]; k < m.colptr[p + 1]; ++k) {
            const int32_t pos = cursor[m.rowidx[k]]++;
            m.indices[pos] = (int32_t)p;
            m.data[pos] = m.cdata[k];
        }
    }
    return AZI_OK;
}

void build_tiles(const int32_t* indptr, int32_t nrows, int64_t z_off, int64_t r_off,
                 int64_t ip_off, int32_t tile_nnz, std::vector<Tile>& tiles,
                 std::vector<Split>& splits, int32_t& nparts) {
    int32_t r = 0;
    while (r < nrows) {
        const int32_t len = indptr[r + 1] - indptr[r];
        if (len > tile_nnz) {
            // Long row: nearly equal pieces, inner cuts on multiples of 4 so
            // the 4-wide loads of a piece do not straddle its neighbour.
            const int32_t pieces = (len + tile_nnz - 1) / tile_nnz;
            const int32_t p0 = nparts;
            int32_t prev = indptr[r];
            for (int32_t k = 0; k < pieces; ++k) {
                int32_t next = indptr[r + 1];
                if (k + 1 < pieces) {
                    next = indptr[r] + (int32_t)(((int64_t)len * (k + 1)) / pieces);
                    next &= ~3;
                    next = std::max(next, prev + 1);
                }
                Tile t{(int32_t)(r_off + r), (int32_t)(r_off + r + 1), (int32_t)(z_off + prev),
                       (int32_t)(z_off + next), nparts++, (int32_t)(ip_off + r), 0, 0};
                tiles.push_back(t);
                prev = next;
            }
            splits.push_back(Split{(int32_t)(r_off + r), p0, nparts, 0});
            ++r;
            continue;
        }
        // Whole rows, as many as fit in tile_nnz nonzeros (rows per tile
        // bounded as well, so a tile of empty rows stays small).
        const int32_t start = r;
        int32_t acc = 0;
        const int32_t max_rows = std::max(tile_nnz / 4, 64);
        while (r < nrows && r - start < max_rows) {
            const int32_t l = indptr[r + 1] - indptr[r];
            if (l > tile_nnz || acc + l > tile_nnz) break;
            acc += l;
            ++r;
        }
        Tile t{(int32_t)(r_off + start), (int32_t)(r_off + r), (int32_t)(z_off + indptr[start]),
               (int32_t)(z_off + indptr[r]), -1, (int32_t)(ip_off + start), 0, 0};
        tiles.push_back(t);
    }
}

}  // namespace azi
