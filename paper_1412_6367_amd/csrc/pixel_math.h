// Per-pixel geometry of the plan builders, shared by the host builder and
// the device builder so that both form every quantity that decides a bin
// index by the same sequence of IEEE operations.  Both translation units are
// compiled without floating-point contraction.
#pragma once

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace azi {

// std::max / std::min semantics, usable on both sides.
template <class T>
__host__ __device__ constexpr T vmax(T a, T b) { return (a < b) ? b : a; }
template <class T>
__host__ __device__ constexpr T vmin(T a, T b) { return (b < a) ? b : a; }

// Output coordinate of a radius r in metres (Section 3 coordinate list):
// 2theta = atan(r / d), q = 4 pi sin(2theta / 2) / lambda with lambda in nm.
__host__ __device__ inline double to_unit(double r, int32_t unit, double dist, double wl) {
    switch (unit) {
        case AZI_UNIT_R_M: return r;
        case AZI_UNIT_R_MM: return r * 1e3;
        default: break;
    }
    const double tth = ::atan(r / dist);
    if (unit == AZI_UNIT_2TH_RAD) return tth;
    if (unit == AZI_UNIT_2TH_DEG) return tth * (180.0 / M_PI);
    return (4.0 * M_PI) * ::sin(tth / 2.0) / (wl * 1e9);
}

// Radial extent of pixel (i, j) = the square [j, j+1] x [i, i+1]: the
// farthest corner and the nearest point of the square from the beam centre
// (the box circumscribing the pixel in the radial direction), and the
// radius of the pixel midpoint.
struct Extent { double lo, hi, mid; };

__host__ __device__ inline Extent pixel_extent(int64_t i, int64_t j, const azi_geom& g) {
    const double cx = g.center_x_px, cy = g.center_y_px;
    const double px = g.pixel_x_m, py = g.pixel_y_m;
    const double x0 = ((double)j - cx) * px, x1 = ((double)(j + 1) - cx) * px;
    const double y0 = ((double)i - cy) * py, y1 = ((double)(i + 1) - cy) * py;
    const double a = x0 * x0, b = x1 * x1, c = y0 * y0, d = y1 * y1;
    const double s = vmax(vmax(a + c, b + c), vmax(a + d, b + d));
    const double ex = vmax(vmax((double)j - cx, cx - (double)(j + 1)), 0.0) * px;
    const double ey = vmax(vmax((double)i - cy, cy - (double)(i + 1)), 0.0) * py;
    const double xm = ((double)j + 0.5 - cx) * px, ym = ((double)i + 0.5 - cy) * py;
    Extent e;
    e.hi = ::sqrt(s);
    e.lo = ::sqrt(ex * ex + ey * ey);
    e.mid = ::sqrt(xm * xm + ym * ym);
    return e;
}

// The entries of one pixel for a box [lo, hi] over bins of width delta from
// pmin: fractional positions fl, fh; the inside part [flc, fhc] of [0, npt];
// bins b0 = floor(flc) .. b1 = ceil(fhc) - 1; weight = overlap / (fh - fl):
// cl for b0 (the only weight when b0 == b1), cr for b1, ci for the bins
// between.  b0 > b1 means no entry; fl tells below the range from above it.
struct BoxTerms {
    int32_t b0, b1;
    double cl, ci, cr, fl;
};

__host__ __device__ inline BoxTerms bbox_terms(double lo, double hi, double pmin, double delta,
                                               int32_t npt) {
    BoxTerms t{1, 0, 0.0, 0.0, 0.0, 0.0};
    const double fl = (lo - pmin) / delta;
    const double fh = (hi - pmin) / delta;
    const double n = (double)npt;
    t.fl = fl;
    if (fh == fl) {  // zero-width box: whole weight to its bin
        if (fl >= 0.0 && fl <= n) {
            t.b0 = t.b1 = vmin((int32_t)::floor(fl), npt - 1);
            t.cl = 1.0;
        }
        return t;
    }
    const double flc = vmax(fl, 0.0);
    const double fhc = vmin(fh, n);
    if (!(fhc > flc)) return t;
    const double width = fh - fl;
    t.b0 = (int32_t)::floor(flc);
    t.b1 = (int32_t)::ceil(fhc) - 1;
    if (t.b0 == t.b1) {
        t.cl = (fhc - flc) / width;
        return t;
    }
    t.cl = ((double)(t.b0 + 1) - flc) / width;
    if (t.b1 > t.b0 + 1) t.ci = 1.0 / width;
    t.cr = (fhc - (double)t.b1) / width;
    return t;
}

template <class Emit>
__host__ __device__ inline void bbox_pixel(double lo, double hi, double pmin, double delta,
                                           int32_t npt, Emit&& emit) {
    const BoxTerms t = bbox_terms(lo, hi, pmin, delta, npt);
    if (t.b0 > t.b1) return;
    emit(t.b0, t.cl);
    if (t.b1 == t.b0) return;
    for (int32_t b = t.b0 + 1; b < t.b1; ++b) emit(b, t.ci);
    emit(t.b1, t.cr);
}

// Full splitting (Section 4.2): the pixel's four corners, mapped to
// (output unit, azimuth) and joined by straight edges, form a
// quadrilateral; bin b gets the part of its area within the bin's slab of
// the output unit over its whole area.  The area within a slab is the sum,
// over the four edges, of the integral of the edge's line over the slab
// (the vertical edges of the clipped polygon add nothing), in absolute
// value.  Coordinates are taken relative to the first corner.
struct Quad { double x[4], y[4]; };

__host__ __device__ inline double edge_integral(const Quad& q, double e0, double e1) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double ax = q.x[k], ay = q.y[k];
        const double bx = q.x[(k + 1) & 3], by = q.y[(k + 1) & 3];
        if (ax == bx) continue;
        const double lo = vmax(vmin(ax, bx), e0);
        const double hi = vmin(vmax(ax, bx), e1);
        if (!(hi > lo)) continue;
        const double slope = (by - ay) / (bx - ax);
        const double ylo = ay + (lo - ax) * slope;
        const double yhi = ay + (hi - ax) * slope;
        const double part = (hi - lo) * (ylo + yhi) / 2.0;
        s += bx > ax ? part : -part;
    }
    return ::fabs(s);
}

template <class Emit>
__host__ __device__ inline void full_pixel(int64_t i, int64_t j, const azi_geom& g, int32_t unit, double lo, double hi,
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
        p0[k] = to_unit(::sqrt(x * x + y * y), unit, g.dist_m, g.wavelength_m);
        p1[k] = ::atan2(y, x);
    }
    for (int k = 1; k < 4; ++k)
        p1[k] += ::nearbyint((p1[0] - p1[k]) / (2.0 * M_PI)) * (2.0 * M_PI);
    const double mn = vmin(vmin(p0[0], p0[1]), vmin(p0[2], p0[3]));
    const double mx = vmax(vmax(p0[0], p0[1]), vmax(p0[2], p0[3]));
    Quad q;
    for (int k = 0; k < 4; ++k) {
        q.x[k] = p0[k] - p0[0];
        q.y[k] = p1[k] - p1[0];
    }
    const double area = edge_integral(q, -HUGE_VAL, HUGE_VAL);
    const double fl = (mn - pmin) / delta, fh = (mx - pmin) / delta;
    if (area == 0.0 || fh == fl) return;
    const int32_t b0 = vmax((int32_t)::floor(fl), 0);
    const int32_t b1 = vmin((int32_t)::ceil(fh) - 1, npt - 1);
    for (int32_t b = b0; b <= b1; ++b) {
        const double e0 = (pmin + b * delta) - p0[0];
        const double e1 = (pmin + (b + 1) * delta) - p0[0];
        const double c = edge_integral(q, e0, e1) / area;
        if (c > 0.0) emit(b, c);
    }
}

// ---------------------------------------------------------------------------
// Two-dimensional integration (radius x azimuth): rows are (wedge k, radial
// bin b) -> k * nrad + b, wedges of width dchi from -pi, periodic.
// ---------------------------------------------------------------------------
struct Grid2d {
    double pmin, delta, dchi;
    int32_t nrad, nazim;
};

__host__ __device__ inline int32_t wrap_wedge(int64_t k, int32_t n) {
    return (int32_t)(((k % n) + n) % n);
}

// Azimuths chi = atan2(y, x) of the four corners of pixel (i, j), in the
// order (j, i), (j+1, i), (j+1, i+1), (j, i+1), unwrapped to within pi of
// the first corner; p0 (optional) receives the corners' output coordinate.
__host__ __device__ inline void pixel_corners(int64_t i, int64_t j, const azi_geom& g,
                                              int32_t unit, double* p0, double* p1) {
    const int da[4] = {0, 1, 1, 0}, db[4] = {0, 0, 1, 1};
    for (int k = 0; k < 4; ++k) {
        const double x = ((double)(j + da[k]) - g.center_x_px) * g.pixel_x_m;
        const double y = ((double)(i + db[k]) - g.center_y_px) * g.pixel_y_m;
        if (p0) p0[k] = to_unit(::sqrt(x * x + y * y), unit, g.dist_m, g.wavelength_m);
        p1[k] = ::atan2(y, x);
    }
    for (int k = 1; k < 4; ++k)
        p1[k] += ::nearbyint((p1[0] - p1[k]) / (2.0 * M_PI)) * (2.0 * M_PI);
}

// Calls f(k) for every raw wedge index k of [k0, k1] in ascending order of
// the wedge it wraps to (ties, possible with very few wedges, by ascending
// k): the pixel's entries then come out in ascending row order.
template <class F>
__host__ __device__ inline void wedges_ascending(int64_t k0, int64_t k1, int32_t n, F&& f) {
    if (k1 < k0) return;
    const int64_t t0 = k0 >= 0 ? k0 / n : -((-k0 + n - 1) / n);  // floor(k / n)
    const int64_t t1 = k1 >= 0 ? k1 / n : -((-k1 + n - 1) / n);
    if (t0 == t1) {
        for (int64_t k = k0; k <= k1; ++k) f(k);
        return;
    }
    if (t1 == t0 + 1 && k1 - k0 + 1 < n) {  // one crossing of the periodic cut
        for (int64_t k = t1 * n; k <= k1; ++k) f(k);
        for (int64_t k = k0; k < t1 * n; ++k) f(k);
        return;
    }
    for (int32_t w = 0; w < n; ++w)
        for (int64_t t = t0; t <= t1; ++t) {
            const int64_t k = w + t * n;
            if (k >= k0 && k <= k1) f(k);
        }
}

// Bounding box in two dimensions: the radial shares of the box (as in one
// dimension) times the azimuthal shares of [chi_lo, chi_hi], the range of
// the corner azimuths (along a straight edge that misses the beam the
// azimuth is monotone): outer wedges get their overlap over the span, inner
// ones 1 / span; a pixel holding the beam spreads evenly over all wedges.
// emit(row, c) in ascending row order.
template <class Emit>
__host__ __device__ inline void bbox2d_entries(int64_t i, int64_t j, const azi_geom& g, double lo,
                                               double hi, const Grid2d& G, Emit&& emit) {
    const BoxTerms rt = bbox_terms(lo, hi, G.pmin, G.delta, G.nrad);
    if (rt.b0 > rt.b1) return;
    auto radial = [&](int32_t w, double ac) {
        const int32_t row0 = w * G.nrad;
        emit(row0 + rt.b0, rt.cl * ac);
        if (rt.b1 == rt.b0) return;
        for (int32_t b = rt.b0 + 1; b < rt.b1; ++b) emit(row0 + b, rt.ci * ac);
        emit(row0 + rt.b1, rt.cr * ac);
    };
    if (lo == 0.0) {
        for (int32_t k = 0; k < G.nazim; ++k) radial(k, 1.0 / G.nazim);
        return;
    }
    double p1[4];
    pixel_corners(i, j, g, AZI_UNIT_R_M, nullptr, p1);
    const double clo = vmin(vmin(p1[0], p1[1]), vmin(p1[2], p1[3]));
    const double chi = vmax(vmax(p1[0], p1[1]), vmax(p1[2], p1[3]));
    const double gl = (clo + M_PI) / G.dchi;
    const double gh = (chi + M_PI) / G.dchi;
    const double width = gh - gl;
    const int64_t k0 = (int64_t)::floor(gl);
    int64_t k1 = (int64_t)::ceil(gh) - 1;
    if (width == 0.0 || k1 < k0) k1 = k0;
    wedges_ascending(k0, k1, G.nazim, [&](int64_t k) {
        double c;
        if (k0 == k1) c = 1.0;
        else if (k == k0) c = ((double)(k0 + 1) - gl) / width;
        else if (k == k1) c = (gh - (double)k1) / width;
        else c = 1.0 / width;
        if (c > 0.0) radial(wrap_wedge(k, G.nazim), c);
    });
}

// Integral over [a, b] of clamp(y0 + (x - x0) * slope, t0, t1): the
// interval is cut where the line meets t0 and t1, and the clamped line is
// linear on every piece, so each piece is an exact trapezoid.
__host__ __device__ inline double clamped_line(double x0, double y0, double slope, double a,
                                               double b, double t0, double t1) {
    double cut[4];
    int n = 0;
    cut[n++] = a;
    if (slope != 0.0) {
        double xa = x0 + (t0 - y0) / slope, xb = x0 + (t1 - y0) / slope;
        if (xa > xb) {
            const double tmp = xa;
            xa = xb;
            xb = tmp;
        }
        if (xa > a && xa < b) cut[n++] = xa;
        if (xb > a && xb < b) cut[n++] = xb;
    }
    cut[n++] = b;
    double s = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        const double u = cut[k], v = cut[k + 1];
        const double yu = vmin(vmax(y0 + (u - x0) * slope, t0), t1);
        const double yv = vmin(vmax(y0 + (v - x0) * slope, t0), t1);
        s += (v - u) * (yu + yv) / 2.0;
    }
    return s;
}

// Area of the quadrilateral inside [e0, e1] x [t0, t1]: over every x of the
// slab, the boundary's lower and upper crossings bound the section, and
// clamp(upper) - clamp(lower) is the part of it inside [t0, t1]; summing the
// clamped edge lines with the edge's direction as sign gives that total.
__host__ __device__ inline double edge_integral_box(const Quad& q, double e0, double e1,
                                                    double t0, double t1) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double ax = q.x[k], ay = q.y[k];
        const double bx = q.x[(k + 1) & 3], by = q.y[(k + 1) & 3];
        if (ax == bx) continue;
        const double lo = vmax(vmin(ax, bx), e0);
        const double hi = vmin(vmax(ax, bx), e1);
        if (!(hi > lo)) continue;
        const double part = clamped_line(ax, ay, (by - ay) / (bx - ax), lo, hi, t0, t1);
        s += bx > ax ? part : -part;
    }
    return ::fabs(s);
}

// Full splitting in two dimensions: the quadrilateral of the corners in
// (output unit, azimuth) clipped to each bin's rectangle, the wedge repeated
// every 2 pi; a pixel holding the beam takes the bounding box.  emit(row, c)
// in ascending row order.
template <class Emit>
__host__ __device__ inline void full2d_entries(int64_t i, int64_t j, const azi_geom& g,
                                               int32_t unit, double lo, double hi,
                                               const Grid2d& G, Emit&& emit) {
    if (lo == 0.0) {
        bbox2d_entries(i, j, g, lo, hi, G, emit);
        return;
    }
    double p0[4], p1[4];
    pixel_corners(i, j, g, unit, p0, p1);
    const double mn = vmin(vmin(p0[0], p0[1]), vmin(p0[2], p0[3]));
    const double mx = vmax(vmax(p0[0], p0[1]), vmax(p0[2], p0[3]));
    const double cmn = vmin(vmin(p1[0], p1[1]), vmin(p1[2], p1[3]));
    const double cmx = vmax(vmax(p1[0], p1[1]), vmax(p1[2], p1[3]));
    Quad q;
    for (int k = 0; k < 4; ++k) {
        q.x[k] = p0[k] - p0[0];
        q.y[k] = p1[k] - p1[0];
    }
    const double area = edge_integral(q, -HUGE_VAL, HUGE_VAL);
    const double fl = (mn - G.pmin) / G.delta, fh = (mx - G.pmin) / G.delta;
    if (area == 0.0 || fh == fl) return;
    const int32_t b0 = vmax((int32_t)::floor(fl), 0);
    const int32_t b1 = vmin((int32_t)::ceil(fh) - 1, G.nrad - 1);
    const int64_t k0 = (int64_t)::floor((cmn + M_PI) / G.dchi);
    const int64_t k1 = vmax((int64_t)::ceil((cmx + M_PI) / G.dchi) - 1, k0);
    wedges_ascending(k0, k1, G.nazim, [&](int64_t k) {
        const double t0 = (-M_PI + (double)k * G.dchi) - p1[0];
        const double t1 = (-M_PI + (double)(k + 1) * G.dchi) - p1[0];
        const int32_t row0 = wrap_wedge(k, G.nazim) * G.nrad;
        for (int32_t b = b0; b <= b1; ++b) {
            const double e0 = (G.pmin + b * G.delta) - p0[0];
            const double e1 = (G.pmin + (b + 1) * G.delta) - p0[0];
            const double c = edge_integral_box(q, e0, e1, t0, t1) / area;
            if (c > 0.0) emit(row0 + b, c);
        }
    });
}

// No split in two dimensions: the bin of the pixel midpoint, fc its
// fractional radial position.
template <class Emit>
__host__ __device__ inline void none2d_entry(int64_t i, int64_t j, const azi_geom& g, double fc,
                                             const Grid2d& G, Emit&& emit) {
    if (!(fc >= 0.0 && fc <= (double)G.nrad)) return;
    const double xc = ((double)j + 0.5 - g.center_x_px) * g.pixel_x_m;
    const double yc = ((double)i + 0.5 - g.center_y_px) * g.pixel_y_m;
    const int64_t k = (int64_t)::floor((::atan2(yc, xc) + M_PI) / G.dchi);
    emit(wrap_wedge(k, G.nazim) * G.nrad + vmin((int32_t)::floor(fc), G.nrad - 1), 1.0);
}

}  // namespace azi
