// Host-only driver of the plan builder for the sanitizer build (AddressSanitizer
// and UndefinedBehaviorSanitizer on g++): builds the matrix of every geometry
// given on stdin, then every host-side layout built from it (ring order,
// staging tiles, image-tile blocks, bands, runs, the matrix-free schedule,
// the CSR tile schedule), checks the invariants the device kernels rely on,
// and prints one line per geometry: "ok <nnz> <runs>", or "err <code>".
//
// Input, one geometry per line:
//   h w center_y center_x npt npt_azim unit split range_min range_max
// (npt_azim 0 for a one-dimensional matrix; range_min > range_max for the
// default range).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1412_6367_amd/csrc/internal.h"

namespace {

int fails = 0;

void expect(bool ok, const char* what, int line) {
    if (!ok) {
        std::fprintf(stderr, "check failed (%s) on geometry %d\n", what, line);
        ++fails;
    }
}

}  // namespace

int main() {
    int h, w, npt, npt_azim, unit, split;
    double cy, cx, rmin, rmax;
    int line = 0;
    while (std::scanf("%d %d %lf %lf %d %d %d %d %lf %lf", &h, &w, &cy, &cx, &npt, &npt_azim,
                      &unit, &split, &rmin, &rmax) == 10) {
        ++line;
        azi_geom g{h, w, 1e-4, 1e-4, cy, cx, 0.1, 1e-10};
        const double range2[2] = {rmin, rmax};
        azi::HostMatrix m;
        std::string err;
        const int rc = azi::build_matrix(g, npt, npt_azim, unit, split,
                                         rmin < rmax ? range2 : nullptr, m, err);
        if (rc != AZI_OK) {
            std::printf("err %d\n", rc);
            continue;
        }
        const int64_t nnz = m.nnz();
        const int64_t npix = m.npix;
        // CSC and CSR describe the same entries, each sorted within its line
        expect((int64_t)m.colptr.size() == npix + 1 && m.colptr[npix] == nnz, "colptr", line);
        expect((int64_t)m.indptr.size() == m.npt + 1 && m.indptr[m.npt] == nnz, "indptr", line);
        std::vector<double> row_sum(m.npt, 0.0), col_row_sum(m.npt, 0.0);
        for (int64_t p = 0; p < npix; ++p)
            for (int32_t k = m.colptr[p]; k < m.colptr[p + 1]; ++k) {
                expect(k == m.colptr[p] || m.rowidx[k] > m.rowidx[k - 1], "csc order", line);
                col_row_sum[m.rowidx[k]] += m.cdata[k];
            }
        for (int32_t b = 0; b < m.npt; ++b)
            for (int32_t k = m.indptr[b]; k < m.indptr[b + 1]; ++k) {
                expect(k == m.indptr[b] || m.indices[k] > m.indices[k - 1], "csr order", line);
                row_sum[b] += m.data[k];
            }
        for (int32_t b = 0; b < m.npt; ++b) expect(row_sum[b] == col_row_sum[b], "row sums", line);

        azi::RingLayout ring;
        azi::build_ring(m, ring);
        std::vector<azi::StageTile> st;
        std::vector<uint16_t> lidx;
        std::vector<int32_t> dest;
        azi::build_stage_tiles(h, w, ring.pos.data(), 0, 0, 0, st, lidx, dest);

        azi::BlockMatrix bm;
        azi::build_blocks(m, h, w, 0, 0, bm);
        azi::finish_blocks(m.npt, bm);
        expect((int64_t)bm.coef.size() == nnz, "block entries", line);

        int64_t runs_total = -1;
        azi::BandMatrix band;
        if (azi::build_bands(m, 4, 512, 0, 0, band)) {
            int64_t entries = 0;
            for (int32_t v : band.packed) entries += v >= 0;
            expect(entries == nnz, "band entries", line);
        }
        azi::RunMatrix rm;
        if (azi::build_runs(m, 1024, 0, 0, rm)) {
            int64_t entries = 0;
            runs_total = 0;
            for (int32_t v : rm.runs)
                if (v >= 0) {
                    entries += ((v >> azi::kRunCountShift) & 3) + 1;
                    ++runs_total;
                }
            expect(entries == nnz && (int64_t)rm.coef.size() >= nnz, "run entries", line);
        }
        // neighbouring bands per workgroup, coefficients scaled per pixel
        std::vector<double> scale((size_t)m.npix, 0.5);
        for (int32_t waves : {4, 8}) {
            azi::RunMatrix rg;
            if (azi::build_runs(m, 256, 0, 0, rg, scale.data(), waves)) {
                expect(rg.pieces.size() % (size_t)waves == 0, "grouped entries", line);
                expect(rg.runs == rm.runs, "grouped runs", line);
                bool halves = rg.coef.size() == rm.coef.size();
                for (size_t k = 0; halves && k < rg.coef.size(); ++k)
                    halves = rg.coef[k] == 0.5 * rm.coef[k];
                expect(halves, "scaled coefficients", line);
            }
        }
        // balanced rounds of 64 and 2048 workgroups: every run in one
        // entry, no band's stretch above 2048 runs unless one group of 64
        // already overflows the rounds
        for (int64_t round : {64, 2048})
            for (int32_t waves : {4, 8}) {
                azi::RunMatrix rb;
                if (!azi::build_runs(m, 4096, 0, 0, rb, nullptr, waves, round)) continue;
                expect(rb.pieces.size() % (size_t)waves == 0, "balanced entries", line);
                int64_t covered = 0, longest = 0;
                for (const azi::BandPiece& pc : rb.pieces)
                    if (pc.slot0 >= 0) {
                        covered += pc.z1 - pc.z0;
                        longest = std::max<int64_t>(longest, pc.z1 - pc.z0);
                    }
                expect(covered == (int64_t)rb.runs.size(), "balanced cover", line);
                expect(longest <= azi::kRoundRuns || longest == 64, "balanced bound", line);
            }
        if (!m.two_d) {
            std::vector<azi::FusedTile> ft;
            std::vector<int32_t> slots, bin_ptr;
            azi::build_fused(m, h, w, ft, slots, bin_ptr);
        }
        for (int32_t tile : {64, 1024, 4096})
            for (int32_t bnd : {1, 4}) {
                std::vector<azi::Tile> tiles;
                std::vector<azi::Split> splits;
                int32_t nparts = 0;
                azi::build_tiles(m.indptr.data(), m.npt, 0, 0, 0, tile, bnd, tiles, splits,
                                 nparts);
            }
        std::printf("ok %lld %lld\n", (long long)nnz, (long long)runs_total);
    }
    std::fflush(stdout);
    return fails ? 1 : 0;
}
