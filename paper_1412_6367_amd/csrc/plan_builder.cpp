// Host plan builder: detector geometry -> per-pixel radial (and azimuthal)
// extent -> bounding-box coefficients (Section 4.1), full-splitting areas
// (Section 4.2) or whole-pixel histogram entries (Section 3.3), in one
// dimension (radius) or two (radius x azimuth) -> pixel-major (CSC) and
// bin-major (CSR, Section 5.2.1) matrices -> tile schedule for the gather
// kernels.
//
// Compiled without floating-point contraction: every quantity that decides
// a bin index is formed by the same sequence of correctly rounded IEEE
// operations (+, -, *, /, sqrt, floor, ceil) as the plain definition, so
// the integer structure of the matrix is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <limits>

#include "internal.h"
#include "pixel_math.h"

namespace azi {
int build_matrix(const azi_geom& g, int32_t npt, int32_t npt_azim, int32_t unit, int32_t split,
                 const double* range2, HostMatrix& m, std::string& err) {
    const int64_t h = g.h, w = g.w, npix = h * w;
    const bool two_d = npt_azim > 0;
    const int32_t nrad = npt;
    if (two_d) {
        if ((int64_t)nrad * npt_azim >= (int64_t)std::numeric_limits<int32_t>::max()) {
            err = "npt_rad * npt_azim is 2^31 or more";
            return AZI_EOVERFLOW;
        }
        npt = nrad * npt_azim;
    }
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
    const double delta = (pmax - pmin) / nrad;
    m.npt = npt;
    m.npt_rad = nrad;
    m.npt_azim = two_d ? npt_azim : 1;
    m.two_d = two_d;
    m.npix = npix;
    m.pmin = pmin;
    m.pmax = pmax;

    // Pixel-major pass: the CSC comes out in pixel order directly.
    m.colptr.assign(npix + 1, 0);
    m.rowidx.clear();
    m.cdata.clear();
    const int64_t limit = std::numeric_limits<int32_t>::max();
    int64_t reserve = boxes ? npix * 3 : npix;
    if (!two_d && split != AZI_SPLIT_FULL) {
        // one-dimensional bounding box or no split: a pixel's entries are
        // exactly the bins b0 .. b1 of its box (never a zero coefficient),
        // so the count is known before anything is stored
        int64_t nnz = 0;
        for (int64_t p = 0; p < npix; ++p) {
            if (split == AZI_SPLIT_BBOX) {
                const BoxTerms t = bbox_terms(lo[p], hi[p], pmin, delta, npt);
                if (t.b0 <= t.b1) nnz += (int64_t)t.b1 - t.b0 + 1;
            } else {
                const double fc = (lo[p] - pmin) / delta;
                if (fc >= 0.0 && fc <= (double)npt) ++nnz;
            }
        }
        if (nnz >= limit) {
            err = "matrix has 2^31 nonzeros or more";
            return AZI_EOVERFLOW;
        }
        reserve = nnz;
    }
    m.rowidx.reserve(reserve);
    m.cdata.reserve(m.rowidx.capacity());
    auto push = [&](int32_t b, double c) {
        m.rowidx.push_back(b);
        m.cdata.push_back(c);
    };
    const Grid2d G{pmin, delta, two_d ? (2.0 * M_PI) / npt_azim : 0.0, nrad, m.npt_azim};
    for (int64_t p = 0; p < npix; ++p) {
        if (two_d) {
            // a pixel's entries come out in ascending row order
            const int64_t i = p / w, j = p % w;
            if (split == AZI_SPLIT_BBOX) bbox2d_entries(i, j, g, lo[p], hi[p], G, push);
            else if (split == AZI_SPLIT_FULL) full2d_entries(i, j, g, unit, lo[p], hi[p], G, push);
            else none2d_entry(i, j, g, (lo[p] - pmin) / delta, G, push);
        } else if (split == AZI_SPLIT_BBOX) {
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
    band_pieces(start.data(), nbands, npt, R, piece_nnz, base, pix_off, bin_off, bm);
    return true;
}

void band_pieces(const int64_t* start, int32_t nbands, int32_t npt, int32_t R, int32_t piece_nnz,
                 int64_t base, int64_t pix_off, int64_t bin_off, BandMatrix& bm) {
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
}

bool build_runs(const HostMatrix& m, int32_t piece_runs, int64_t pix_off, int64_t bin_off,
                RunMatrix& rm, const double* scale, int32_t waves, int64_t round_tiles) {
    constexpr int32_t R = kRunRows;
    if (m.npix >= ((int64_t)1 << kBandShift)) return false;
    const int32_t npt = m.npt;
    const int32_t nbands = (npt + R - 1) / R;
    // runs: maximal stretches of a pixel's entries in one band with
    // consecutive bins (every stretch of a one-dimensional plan)
    auto for_runs = [&](auto&& f) {
        for (int64_t p = 0; p < m.npix; ++p) {
            int32_t k = m.colptr[p];
            const int32_t k1 = m.colptr[p + 1];
            while (k < k1) {
                int32_t e = k + 1;
                while (e < k1 && m.rowidx[e] == m.rowidx[e - 1] + 1 &&
                       m.rowidx[e] / R == m.rowidx[k] / R)
                    ++e;
                f(p, k, e);
                k = e;
            }
        }
    };
    std::vector<int64_t> cnt(nbands, 0);
    for_runs([&](int64_t, int32_t k, int32_t) { cnt[m.rowidx[k] / R]++; });
    // this instance's runs begin at the (64-aligned) end of rm.runs
    const int64_t base = (int64_t)rm.runs.size();
    std::vector<int64_t> start(nbands + 1, base);
    for (int32_t b = 0; b < nbands; ++b) start[b + 1] = start[b] + (cnt[b] + 63) / 64 * 64;
    if (start[nbands] >= (int64_t)INT32_MAX ||
        (int64_t)rm.coef.size() + m.nnz() >= (int64_t)INT32_MAX)
        return false;
    rm.runs.resize(start[nbands], -1);  // padding to the next band: no run
    std::vector<int32_t> first_k(start[nbands] - base, 0);  // CSC position of a run's first entry
    std::vector<int64_t> cur(start.begin(), start.end() - 1);
    for_runs([&](int64_t p, int32_t k, int32_t e) {
        const int32_t b = m.rowidx[k];
        const int64_t z = cur[b / R]++;
        rm.runs[z] = (int32_t)p | ((b % R) << kBandShift) | ((e - k - 1) << kRunCountShift);
        first_k[z - base] = k;
    });
    // coefficients, slot-major per group of 64 runs (group = run index / 64)
    rm.gbase.resize(start[nbands] / 64, 0);
    int64_t pos = (int64_t)rm.coef.size();
    rm.coef.resize(pos + m.nnz(), 0.0);
    for (int32_t b = 0; b < nbands; ++b) {
        for (int64_t g = start[b] / 64; g < start[b + 1] / 64; ++g) {
            rm.gbase[g] = (int32_t)pos;
            const int64_t z0 = g * 64, z1 = std::min(z0 + 64, start[b] + cnt[b]);
            for (int32_t j = 0; j < R; ++j)
                for (int64_t z = z0; z < z1; ++z)
                    if ((rm.runs[z] >> kRunCountShift) + 1 > j) {
                        const double c = m.cdata[first_k[z - base] + j];
                        rm.coef[pos++] =
                            scale ? c * scale[rm.runs[z] & ((1 << kBandShift) - 1)] : c;
                    }
        }
    }
    // pieces: each band cut into near-equal parts on multiples of 64 runs
    if (rm.bin_slot.size() < (size_t)(bin_off + npt)) {
        rm.bin_slot.resize(bin_off + npt, 0);
        rm.bin_count.resize(bin_off + npt, 0);
    }
    const int64_t chunk = std::max<int64_t>(64, piece_runs / 64 * 64);
    if (waves > 32) return false;  // the stretch counters below hold 32 bands
    if (waves > 1) {
        constexpr int32_t kPixMask = (1 << kBandShift) - 1;
        const int32_t ngroups = (nbands + waves - 1) / waves;
        // Per group of bands, the groups of 64 runs of its bands as events
        // (first pixel, band in the group), in pixel order.
        struct Event {
            int64_t pix;
            int32_t w;
        };
        std::vector<int64_t> ev_off((size_t)ngroups + 1, 0);
        for (int32_t gi = 0; gi < ngroups; ++gi) {
            int64_t n = 0;
            for (int32_t b = gi * waves; b < std::min(nbands, (gi + 1) * waves); ++b)
                n += (cnt[b] + 63) / 64;
            ev_off[gi + 1] = ev_off[gi] + n;
        }
        std::vector<Event> ev((size_t)ev_off[ngroups]);
        for (int32_t gi = 0; gi < ngroups; ++gi) {
            int64_t e = ev_off[gi];
            for (int32_t b = gi * waves; b < std::min(nbands, (gi + 1) * waves); ++b)
                for (int64_t j = 0; j < (cnt[b] + 63) / 64; ++j)
                    ev[e++] = Event{rm.runs[start[b] + 64 * j] & kPixMask, b - gi * waves};
            std::stable_sort(ev.begin() + ev_off[gi], ev.begin() + ev_off[gi + 1],
                             [](const Event& a, const Event& b) { return a.pix < b.pix; });
        }
        // Greedy stretches of group gi in pixel order, none holding more
        // than `bound` groups of 64 runs of one band (events of one pixel stay
        // together); their count, and the first pixel of each stretch but
        // the first in *cuts.
        auto stretches = [&](int32_t gi, int64_t bound, std::vector<int64_t>* cuts) {
            int64_t c[32] = {0};
            int32_t k = 1;
            for (int64_t i = ev_off[gi]; i < ev_off[gi + 1];) {
                int64_t j = i;
                int64_t add[32] = {0};
                while (j < ev_off[gi + 1] && ev[j].pix == ev[i].pix) add[ev[j++].w]++;
                bool over = false;
                for (int32_t w = 0; w < waves; ++w) over |= add[w] > 0 && c[w] + add[w] > bound;
                if (over) {
                    ++k;
                    if (cuts) cuts->push_back(ev[i].pix);
                    for (int32_t w = 0; w < waves; ++w) c[w] = 0;
                }
                for (int32_t w = 0; w < waves; ++w) c[w] += add[w];
                i = j;
            }
            return k;
        };
        int64_t maxg = 1;
        for (int32_t b = 0; b < nbands; ++b) maxg = std::max(maxg, (cnt[b] + 63) / 64);
        // the smallest bound that keeps the schedule within max_tiles workgroups
        auto bound_for = [&](int64_t max_tiles) {
            int64_t lo = 1, hi = maxg;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                int64_t tiles = 0;
                for (int32_t gi = 0; gi < ngroups && tiles <= max_tiles; ++gi)
                    tiles += stretches(gi, mid, nullptr);
                if (tiles <= max_tiles) hi = mid;
                else lo = mid + 1;
            }
            return lo;
        };
        // the bound on a band's groups per stretch: from the piece size, or
        // for rounds of round_tiles workgroups, the fewest rounds whose
        // bound keeps a band's stretch within kRoundRuns runs
        int64_t bound = std::min(maxg, chunk / 64);
        if (round_tiles > 0) {
            for (int64_t k = 1;; ++k) {
                bound = bound_for(k * round_tiles);
                if (bound * 64 <= kRoundRuns || bound == 1) break;
            }
        }
        for (int32_t gi = 0; gi < ngroups; ++gi) {
            const int32_t g0 = gi * waves;
            const int32_t gn = std::min(waves, nbands - g0);
            // as many stretches as the bound needs, each group's as even as
            // that count allows: the smallest bound giving no more
            const int32_t K = stretches(gi, bound, nullptr);
            int64_t lo = 1, hi = bound;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (stretches(gi, mid, nullptr) <= K) hi = mid;
                else lo = mid + 1;
            }
            std::vector<int64_t> cut;
            cut.reserve((size_t)K + 1);
            cut.push_back(0);
            stretches(gi, lo, &cut);
            cut.push_back(std::numeric_limits<int64_t>::max());
            // per band: group boundaries of the stretches (a band's group
            // belongs to the stretch holding its first pixel)
            std::vector<int64_t> zc((size_t)gn * (K + 1));
            for (int32_t w = 0; w < gn; ++w) {
                const int32_t b = g0 + w;
                const int64_t ng = (cnt[b] + 63) / 64;
                int64_t j = 0;
                zc[(size_t)w * (K + 1)] = start[b];
                for (int32_t k = 1; k <= K; ++k) {
                    while (j < ng && (k == K || (rm.runs[start[b] + 64 * j] & kPixMask) < cut[k]))
                        ++j;
                    zc[(size_t)w * (K + 1) + k] = start[b] + 64 * j;
                }
                const int32_t bin0 = b * R;
                const int32_t nrows = std::min(R, npt - bin0);
                for (int32_t r = 0; r < nrows; ++r) {
                    rm.bin_slot[bin_off + bin0 + r] = rm.nslots + w * K * R + r;
                    rm.bin_count[bin_off + bin0 + r] = K;
                }
            }
            for (int32_t k = 0; k < K; ++k) {
                for (int32_t w = 0; w < waves; ++w) {
                    if (w >= gn) {
                        rm.pieces.push_back(BandPiece{0, 0, 0, 0, -1, 0, pix_off});
                        continue;
                    }
                    const int32_t b = g0 + w;
                    const int32_t bin0 = b * R;
                    rm.pieces.push_back(BandPiece{(int32_t)zc[(size_t)w * (K + 1) + k],
                                                  (int32_t)zc[(size_t)w * (K + 1) + k + 1],
                                                  (int32_t)(bin_off + bin0),
                                                  std::min(R, npt - bin0),
                                                  rm.nslots + (w * K + k) * R, 0, pix_off});
                }
            }
            rm.nslots += gn * K * R;
        }
        return true;
    }
    for (int32_t band = 0; band < nbands; ++band) {
        const int32_t bin0 = band * R;
        const int32_t nrows = std::min(R, npt - bin0);
        const int64_t z0 = start[band], len = cnt[band];
        const int32_t pieces = len > 0 ? (int32_t)((len + chunk - 1) / chunk) : 1;
        for (int32_t r = 0; r < nrows; ++r) {
            rm.bin_slot[bin_off + bin0 + r] = rm.nslots + r;
            rm.bin_count[bin_off + bin0 + r] = pieces;
        }
        const int64_t groups = (len + 63) / 64;
        int64_t prev = z0;
        for (int32_t k = 0; k < pieces; ++k) {
            const int64_t next = k + 1 < pieces ? z0 + groups * (k + 1) / pieces * 64 : z0 + len;
            rm.pieces.push_back(BandPiece{(int32_t)prev, (int32_t)next, (int32_t)(bin_off + bin0),
                                          nrows, rm.nslots, 0, pix_off});
            rm.nslots += R;
            prev = next;
        }
    }
    return true;
}

void build_fused(const HostMatrix& m, int32_t h, int32_t w, std::vector<FusedTile>& tiles,
                 std::vector<int32_t>& slots, std::vector<int32_t>& bin_ptr) {
    tiles.clear();
    slots.clear();
    bin_ptr.assign((size_t)m.npt + 1, 0);
    for (int32_t i0 = 0; i0 < h; i0 += kFusedH) {
        const int32_t th = std::min(kFusedH, h - i0);
        for (int32_t j0 = 0; j0 < w; j0 += kFusedW) {
            const int32_t tw = std::min(kFusedW, w - j0);
            int32_t lo = std::numeric_limits<int32_t>::max(), hi = -1;
            for (int32_t r = 0; r < th; ++r) {
                for (int32_t c = 0; c < tw; ++c) {
                    const int64_t p = (int64_t)(i0 + r) * w + j0 + c;
                    if (m.colptr[p] < m.colptr[p + 1]) {
                        lo = std::min(lo, m.rowidx[m.colptr[p]]);
                        hi = std::max(hi, m.rowidx[m.colptr[p + 1] - 1]);
                    }
                }
            }
            FusedTile t{i0, j0, th, tw, 0, 0, 0};
            if (hi >= lo) {
                t.wlo = lo;
                t.nwin = hi - lo + 1;
                for (int32_t b = lo; b <= hi; ++b) bin_ptr[b + 1]++;
            }
            tiles.push_back(t);
        }
    }
    for (int32_t b = 0; b < m.npt; ++b) bin_ptr[b + 1] += bin_ptr[b];
    std::vector<int32_t> cur(bin_ptr.begin(), bin_ptr.end() - 1);
    for (FusedTile& t : tiles) {
        t.slot_off = (int64_t)slots.size();
        for (int32_t k = 0; k < t.nwin; ++k) slots.push_back(cur[t.wlo + k]++);
    }
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
