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

// Full splitting (Section 4.2): the pixel's four corners, mapped to
// (output unit, azimuth) and joined by straight edges, form a
// quadrilateral; bin b gets the part of its area within the bin's slab of
// the output unit over its whole area.  The area within a slab is the sum,
// over the four edges, of the integral of the edge's line over the slab
// (the vertical edges of the clipped polygon add nothing), in absolute
// value.  Coordinates are taken relative to the first corner.
struct Quad { double x[4], y[4]; };

inline double edge_integral(const Quad& q, double e0, double e1) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double ax = q.x[k], ay = q.y[k];
        const double bx = q.x[(k + 1) & 3], by = q.y[(k + 1) & 3];
        if (ax == bx) continue;
        const double lo = std::max(std::min(ax, bx), e0);
        const double hi = std::min(std::max(ax, bx), e1);
        if (!(hi > lo)) continue;
        const double slope = (by - ay) / (bx - ax);
        const double ylo = ay + (lo - ax) * slope;
        const double yhi = ay + (hi - ax) * slope;
        const double part = (hi - lo) * (ylo + yhi) / 2.0;
        s += bx > ax ? part : -part;
    }
    return std::fabs(s);
}

template <class Emit>
inline void full_pixel(int64_t i, int64_t j, const azi_geom& g, int32_t unit, double lo, double hi,
                       double pmin, double delta, int32_t npt, Emit&& emit) {
    if (lo == 0.0) {  // the beam centre lies on this pixel
        bbox_pixel(lo, hi, pmin, delta, npt, emit);
        return;
    }
    const int da[4] = {0, 1, 1, 0}, db[4] = {0, 0, 1, 1};
    double p0[4], p1[4];
    for (int k = 0; k < 4; ++k) {
        const double x = ((double)(j + da[k]) - g.center_x_px) * g.pixel_x_m;
        const double y = ((double)(i + db[k]) - g.center_y_px) * g.pixel_y_m;
        p0[k] = to_unit(std::sqrt(x * x + y * y), unit, g.dist_m, g.wavelength_m);
        p1[k] = std::atan2(y, x);
    }
    for (int k = 1; k < 4; ++k)
        p1[k] += std::nearbyint((p1[0] - p1[k]) / (2.0 * M_PI)) * (2.0 * M_PI);
    const double mn = std::min(std::min(p0[0], p0[1]), std::min(p0[2], p0[3]));
    const double mx = std::max(std::max(p0[0], p0[1]), std::max(p0[2], p0[3]));
    Quad q;
    for (int k = 0; k < 4; ++k) {
        q.x[k] = p0[k] - p0[0];
        q.y[k] = p1[k] - p1[0];
    }
    const double area = edge_integral(q, -HUGE_VAL, HUGE_VAL);
    const double fl = (mn - pmin) / delta, fh = (mx - pmin) / delta;
    if (area == 0.0 || fh == fl) return;
    const int32_t b0 = std::max((int32_t)std::floor(fl), 0);
    const int32_t b1 = std::min((int32_t)std::ceil(fh) - 1, npt - 1);
    for (int32_t b = b0; b <= b1; ++b) {
        const double e0 = (pmin + b * delta) - p0[0];
        const double e1 = (pmin + (b + 1) * delta) - p0[0];
        const double c = edge_integral(q, e0, e1) / area;
        if (c > 0.0) emit(b, c);
    }
}

}  // namespace

int build_matrix(const azi_geom& g, int32_t npt, int32_t unit, int32_t split,
                 const double* range2, HostMatrix& m, std::string& err) {
    const int64_t h = g.h, w = g.w, npix = h * w;
    if (npix >= (int64_t)std::numeric_limits<int32_t>::max()) {
        err = "image has 2^31 pixels or more";
        return AZI_EOVERFLOW;
    }
    const bool boxes = split == AZI_SPLIT_BBOX || split == AZI_SPLIT_FULL;
    std::vector<double> lo, hi;
    if (boxes) { lo.resize(npix); hi.resize(npix); }
    else { lo.resize(npix); }  // pixel-midpoint values
    double mn = std::numeric_limits<double>::infinity(), mx = -mn;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < w; ++j) {
            const int64_t p = i * w + j;
            const Extent e = pixel_extent(i, j, g);
            if (boxes) {
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
    m.rowidx.reserve(boxes ? npix * 3 : npix);
    m.cdata.reserve(m.rowidx.capacity());
    const int64_t limit = std::numeric_limits<int32_t>::max();
    auto push = [&](int32_t b, double c) {
        m.rowidx.push_back(b);
        m.cdata.push_back(c);
    };
    for (int64_t p = 0; p < npix; ++p) {
        if (split == AZI_SPLIT_BBOX) {
            bbox_pixel(lo[p], hi[p], pmin, delta, npt, push);
        } else if (split == AZI_SPLIT_FULL) {
            full_pixel(p / w, p % w, g, unit, lo[p], hi[p], pmin, delta, npt, push);
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

void build_ring(const HostMatrix& m, RingLayout& r) {
    const int64_t npix = m.npix;
    const int32_t npt = m.npt;
    // counting sort of pixels by first bin (pixels feeding no bin go last)
    std::vector<int64_t> start(npt + 2, 0);
    for (int64_t p = 0; p < npix; ++p) {
        const int32_t key = m.colptr[p] < m.colptr[p + 1] ? m.rowidx[m.colptr[p]] : npt;
        start[key + 1]++;
    }
    for (int32_t b = 0; b <= npt; ++b) start[b + 1] += start[b];
    r.used = start[npt];
    r.order.assign(npix, 0);
    r.pos.assign(npix, 0);
    for (int64_t p = 0; p < npix; ++p) {
        const int32_t key = m.colptr[p] < m.colptr[p + 1] ? m.rowidx[m.colptr[p]] : npt;
        r.pos[p] = (int32_t)start[key];
        r.order[start[key]++] = (int32_t)p;
    }
    // rows in ring order: visiting positions in ascending order keeps each
    // row's positions ascending
    const int64_t nnz = m.nnz();
    r.indices.assign(nnz, 0);
    r.data.assign(nnz, 0.0);
    std::vector<int32_t> cursor(m.indptr.begin(), m.indptr.end() - 1);
    for (int64_t q = 0; q < npix; ++q) {
        const int32_t p = r.order[q];
        for (int32_t k = m.colptr[p]; k < m.colptr[p + 1]; ++k) {
            const int32_t pos = cursor[m.rowidx[k]]++;
            r.indices[pos] = (int32_t)q;
            r.data[pos] = m.cdata[k];
        }
    }
}

void build_stage_tiles(int32_t h, int32_t w, const int32_t* pos, int64_t img_off, int64_t q_off,
                       int64_t k_off, std::vector<StageTile>& tiles, std::vector<uint16_t>& lidx,
                       std::vector<int32_t>& dest) {
    std::vector<int32_t> key;
    std::vector<int32_t> perm;
    for (int32_t i0 = 0; i0 < h; i0 += kStageTileH) {
        const int32_t th = std::min(kStageTileH, h - i0);
        for (int32_t j0 = 0; j0 < w; j0 += kStageTileW) {
            const int32_t tw = std::min(kStageTileW, w - j0);
            const int32_t n = th * tw;
            key.resize(n);
            perm.resize(n);
            for (int32_t e = 0; e < n; ++e) {
                const int64_t p = (int64_t)(i0 + e / tw) * w + (j0 + e % tw);
                key[e] = pos[p];
                perm[e] = e;
            }
            std::sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
            const size_t base = lidx.size();
            lidx.resize(base + n);
            dest.resize(base + n);
            for (int32_t k = 0; k < n; ++k) {
                lidx[base + perm[k]] = (uint16_t)k;
                dest[base + k] = (int32_t)(key[perm[k]] + q_off);
            }
            tiles.push_back(StageTile{i0, j0, th, tw, w, 0, img_off, k_off + (int64_t)base});
        }
    }
}

void build_blocks(const HostMatrix& m, int32_t h, int32_t w, int64_t img_off, int64_t bin_off,
                  BlockMatrix& bm) {
    struct Ent { int32_t bin; uint16_t lp; double c; };
    std::vector<Ent> ents;
    for (int32_t i0 = 0; i0 < h; i0 += kStageTileH) {
        const int32_t th = std::min(kStageTileH, h - i0);
        for (int32_t j0 = 0; j0 < w; j0 += kStageTileW) {
            const int32_t tw = std::min(kStageTileW, w - j0);
            ents.clear();
            for (int32_t e = 0; e < th * tw; ++e) {
                const int64_t p = (int64_t)(i0 + e / tw) * w + (j0 + e % tw);
                for (int32_t k = m.colptr[p]; k < m.colptr[p + 1]; ++k)
                    ents.push_back(Ent{m.rowidx[k], (uint16_t)e, m.cdata[k]});
            }
            // rows in ascending bin order, entries of a row in pixel order
            std::stable_sort(ents.begin(), ents.end(),
                             [](const Ent& a, const Ent& b) { return a.bin < b.bin; });
            BlockTile t{i0, j0, th, tw, w, 0, img_off, (int64_t)bm.rows.size(),
                        (int64_t)bm.lp.size()};
            int32_t k = 0;
            const int32_t n = (int32_t)ents.size();
            while (k < n) {
                int32_t e = k;
                while (e < n && ents[e].bin == ents[k].bin) ++e;
                // slot filled in by finish_blocks; keep the bin for now
                bm.rows.push_back(BlockRow{-1, k, e, (int32_t)(ents[k].bin + bin_off)});
                ++t.nrows;
                k = e;
            }
            for (const Ent& en : ents) {
                bm.lp.push_back(en.lp);
                bm.coef.push_back(en.c);
            }
            bm.tiles.push_back(t);
        }
    }
}

void finish_blocks(int64_t npt_total, BlockMatrix& bm) {
    bm.bin_ptr.assign(npt_total + 1, 0);
    for (const BlockRow& r : bm.rows) bm.bin_ptr[r.bin + 1]++;
    for (int64_t b = 0; b < npt_total; ++b) bm.bin_ptr[b + 1] += bm.bin_ptr[b];
    std::vector<int32_t> cursor(bm.bin_ptr.begin(), bm.bin_ptr.end() - 1);
    // rows are stored tile by tile, so slots of a bin follow tile order
    for (BlockRow& r : bm.rows) r.slot = cursor[r.bin]++;
}

bool build_bands(const HostMatrix& m, int32_t R, int32_t piece_nnz, int64_t pix_off,
                 int64_t bin_off, BandMatrix& bm) {
    if (m.npix >= ((int64_t)1 << kBandShift)) return false;
    const int32_t npt = m.npt;
    const int32_t nbands = (npt + R - 1) / R;
    // counting sort of the CSC entries by band; pixels ascending keeps each
    // band's entries in (pixel, bin) order
    std::vector<int64_t> start(nbands + 1, 0);
    for (int64_t k = 0; k < m.nnz(); ++k) start[m.rowidx[k] / R + 1]++;
    for (int32_t b = 0; b < nbands; ++b) start[b + 1] += start[b];
    // instance entries begin on a multiple of 64 of the flat arrays
    while (bm.packed.size() % 64) {
        bm.packed.push_back(0);
        bm.coef.push_back(0.0);
    }
    const int64_t base = (int64_t)bm.packed.size();
    bm.packed.resize(base + m.nnz());
    bm.coef.resize(base + m.nnz());
    std::vector<int64_t> cur(start.begin(), start.end() - 1);
    for (int64_t p = 0; p < m.npix; ++p) {
        for (int32_t k = m.colptr[p]; k < m.colptr[p + 1]; ++k) {
            const int32_t b = m.rowidx[k];
            const int64_t z = base + cur[b / R]++;
            bm.packed[z] = ((b % R) << kBandShift) | (int32_t)p;
            bm.coef[z] = m.cdata[k];
        }
    }
    if (bm.bin_slot.size() < (size_t)(bin_off + npt)) {
        bm.bin_slot.resize(bin_off + npt, 0);
        bm.bin_count.resize(bin_off + npt, 0);
    }
    for (int32_t band = 0; band < nbands; ++band) {
        const int32_t bin0 = band * R;
        const int32_t nrows = std::min(R, npt - bin0);
        const int64_t z0 = base + start[band], z1 = base + start[band + 1];
        const int64_t len = z1 - z0;
        const int32_t pieces = len > 0 ? (int32_t)((len + piece_nnz - 1) / piece_nnz) : 1;
        for (int32_t r = 0; r < nrows; ++r) {
            bm.bin_slot[bin_off + bin0 + r] = bm.nslots + r;
            bm.bin_count[bin_off + bin0 + r] = pieces;
        }
        int64_t prev = z0;
        for (int32_t k = 0; k < pieces; ++k) {
            int64_t next = z1;
            if (k + 1 < pieces) next = std::max(prev + 1, (z0 + len * (k + 1) / pieces) & ~(int64_t)3);
            bm.pieces.push_back(BandPiece{(int32_t)prev, (int32_t)next, (int32_t)(bin_off + bin0),
                                          nrows, bm.nslots, 0, pix_off});
            bm.nslots += R;
            prev = next;
        }
    }
    return true;
}

void build_tiles(const int32_t* indptr, int32_t nrows, int64_t z_off, int64_t r_off,
                 int64_t ip_off, int32_t tile_nnz, int32_t band, std::vector<Tile>& tiles,
                 std::vector<Split>& splits, int32_t& nparts) {
    auto len = [&](int32_t r) { return indptr[r + 1] - indptr[r]; };
    const int32_t R = std::max(band, 1);
    const int32_t inter_min = R > 1 ? tile_nnz / R : INT32_MAX;
    int32_t r = 0;
    while (r < nrows) {
        if (R > 1 && len(r) > inter_min) {
            // a run of up to R consecutive rows, each longer than tile_nnz / R
            int32_t r_end = r + 1;
            int32_t most = len(r);
            while (r_end < nrows && r_end - r < R && len(r_end) > inter_min) {
                most = std::max(most, len(r_end));
                ++r_end;
            }
            const int32_t nr = r_end - r;
            const int64_t total = (int64_t)most * nr;
            int32_t pieces = (int32_t)((total + tile_nnz - 1) / tile_nnz);
            pieces = std::max(1, std::min(pieces, std::max(1, most / 4)));
            const int32_t base = pieces > 1 ? nparts : -1;
            if (pieces > 1) {
                for (int32_t i = 0; i < nr; ++i)
                    splits.push_back(Split{(int32_t)(r_off + r + i), nparts + i * pieces,
                                           nparts + (i + 1) * pieces, 0});
                nparts += nr * pieces;
            }
            for (int32_t k = 0; k < pieces; ++k)
                tiles.push_back(Tile{(int32_t)(r_off + r), (int32_t)(r_off + r_end), 0, pieces,
                                     base, (int32_t)(ip_off + r), kTileInterleave, k});
            r = r_end;
            continue;
        }
        if (len(r) > tile_nnz) {
            // one long row: nearly equal pieces
            const int32_t pieces = (len(r) + tile_nnz - 1) / tile_nnz;
            const int32_t p0 = nparts;
            for (int32_t k = 0; k < pieces; ++k)
                tiles.push_back(Tile{(int32_t)(r_off + r), (int32_t)(r_off + r + 1),
                                     (int32_t)(z_off + piece_cut(indptr[r], indptr[r + 1], k, pieces)),
                                     (int32_t)(z_off + piece_cut(indptr[r], indptr[r + 1], k + 1, pieces)),
                                     nparts++, (int32_t)(ip_off + r), kTileRow, 0});
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
            const int32_t l = len(r);
            if (l > tile_nnz || acc + l > tile_nnz) break;
            if (R > 1 && l > inter_min && r > start) break;  // leave it to an interleave run
            acc += l;
            ++r;
        }
        tiles.push_back(Tile{(int32_t)(r_off + start), (int32_t)(r_off + r),
                             (int32_t)(z_off + indptr[start]), (int32_t)(z_off + indptr[r]), -1,
                             (int32_t)(ip_off + start), r - start == 1 ? kTileRow : kTileRows, 0});
    }
}

}  // namespace azi
