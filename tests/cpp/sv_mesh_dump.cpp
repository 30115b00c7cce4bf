// Writes the library's Scott-Vogelius (Alfeld-refined) mesh of the unit
// square with N cells per side, built on the host, for tests/test_sv_host.py:
// counts, node coordinates, element connectivity, Dirichlet flags, and the
// transfers of the pressure hierarchy (unrefined triangles -> discontinuous
// pressure space, vertex grid -> unrefined triangles) applied to x + 2y.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>
#include "common.h"
namespace mhd { void set_error(const std::string& s) { fprintf(stderr, "%s\n", s.c_str()); } }
using namespace mhd;
int main(int argc, char** argv) {
    if (argc < 3) return 2;
    mhd_mesh_desc d{MHD_MESH_UNIT_SQUARE, atoi(argv[1]), 0, MHD_ELEMENT_SCOTT_VOGELIUS};
    HostMesh m;
    if (build_mesh(&d, m, true) != MHD_OK) return 1;
    FILE* f = fopen(argv[2], "wb");
    if (!f) return 1;
    const int64_t head[6] = {m.nP2, m.nP1, m.n_el, (int64_t)m.levels.size(), m.pin, m.A.nnz()};
    fwrite(head, sizeof(int64_t), 6, f);
    fwrite(m.xy.data(), sizeof(double), m.xy.size(), f);
    fwrite(m.tri.data(), sizeof(int32_t), m.tri.size(), f);
    fwrite(m.dir.data(), 1, m.dir.size(), f);
    // level 1 -> 0: x + 2y given on the unrefined triangles' vertices (unknown 3E + q
    // at vertex q of triangle E, that is vertex 0 of element 3E + q)
    std::vector<double> pv(m.nP1, 0.0), pv1(m.nP1 / 3, 0.0);
    auto lin = [&](int32_t node) { return m.xy[2 * node] + 2.0 * m.xy[2 * node + 1]; };
    if (m.levels.size() > 1) {
        const HostLevel& F = m.levels[0];
        std::vector<double> xc(m.levels[1].n);
        for (int c = 0; c < m.levels[1].n; ++c) xc[c] = lin(m.tri[(size_t)c * 6]);
        for (int64_t r = 0; r < F.P.nrows; ++r)
            for (int32_t p = F.P.rowptr[r]; p < F.P.rowptr[r + 1]; ++p) pv[r] += F.P.val[p] * xc[F.P.col[p]];
    }
    // vertex grid -> level 1: x + 2y on the (N+1)^2 vertices, row-major
    if (m.levels.size() > 2) {
        const HostLevel& F = m.levels[1];
        const HostLevel& C = m.levels[2];
        std::vector<double> xc(C.n);
        for (int k = 0; k <= C.ny; ++k)
            for (int i = 0; i <= C.nx; ++i) xc[(size_t)k * (C.nx + 1) + i] = (i + 2.0 * k) * C.h;
        for (int64_t r = 0; r < F.P.nrows; ++r)
            for (int32_t p = F.P.rowptr[r]; p < F.P.rowptr[r + 1]; ++p) pv1[r] += F.P.val[p] * xc[F.P.col[p]];
    }
    fwrite(pv.data(), sizeof(double), pv.size(), f);
    fwrite(pv1.data(), sizeof(double), pv1.size(), f);
    fclose(f);
    return 0;
}
