// Host side of libmhd_ens: structured triangulations, Taylor-Hood P2/P1
// numbering, CSR patterns of the saddle-point operator, deterministic
// element-to-slot gather lists, the pressure multigrid hierarchy and the
// reference-element tables.  Pure integer/geometry work done once per mesh.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace mhd {

namespace {

// Which square cells of the cell grid belong to the domain.
struct CellDomain {
    int kind;
    int per_unit;   // cells per unit length (step channel); N for the unit square
    bool kept(int i, int k) const {
        if (kind == MHD_MESH_STEP_CHANNEL) return !(i < per_unit && k < per_unit);
        return true;
    }
};

struct Grid {
    int nx, ny;
    double h, x0, y0;
    CellDomain dom;
    bool cell(int i, int k) const {
        if (i < 0 || k < 0 || i >= nx || k >= ny) return false;
        return dom.kept(i, k);
    }
    // vertex (i,k) is active if any of its 4 cells is kept
    int vertex_cells(int i, int k) const {
        return (int)cell(i - 1, k - 1) + (int)cell(i, k - 1) + (int)cell(i - 1, k) + (int)cell(i, k);
    }
};

// the pressure hierarchy stops at a level of at most this many vertices, which
// is solved with its dense inverse (33 x 33 vertices of a unit-square level)
constexpr int kCoarseMax = 1100;
// largest coarsest level whose dense inverse is built (host Gauss-Jordan, about 20 s at 3000)
constexpr int kCoarseDenseMax = 3000;

Grid make_grid(const mhd_mesh_desc* d, int level) {
    Grid g{};
    int s = 1 << level;
    if (d->kind == MHD_MESH_UNIT_SQUARE) {
        g.nx = g.ny = d->nx / s;
        g.h = 1.0 / g.nx;
        g.dom = {d->kind, g.nx};
    } else {
        int m = d->nx / s;
        g.nx = 30 * m;
        g.ny = 10 * m;
        g.h = 1.0 / m;
        g.dom = {d->kind, m};
    }
    g.x0 = g.y0 = 0.0;
    return g;
}

// P1 vertex numbering of a grid: row-major over active vertices.
std::vector<int32_t> vertex_ids(const Grid& g, int& count) {
    std::vector<int32_t> id((size_t)(g.nx + 1) * (g.ny + 1), -1);
    count = 0;
    for (int k = 0; k <= g.ny; ++k)
        for (int i = 0; i <= g.nx; ++i)
            if (g.vertex_cells(i, k) > 0) id[(size_t)k * (g.nx + 1) + i] = count++;
    return id;
}

void grad_bary(const double* p0, const double* p1, const double* p2, double gl[3][2], double& area) {
    double two_a = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]);
    const double* p[3] = {p0, p1, p2};
    for (int i = 0; i < 3; ++i) {
        const double* a = p[(i + 1) % 3];
        const double* b = p[(i + 2) % 3];
        gl[i][0] = (a[1] - b[1]) / two_a;
        gl[i][1] = (b[0] - a[0]) / two_a;
    }
    area = 0.5 * std::fabs(two_a);
}

// rows of (row, col, val) triplets -> CSR with summed duplicates, sorted columns
HostCSR triplets_to_csr(int64_t nrows, int64_t ncols, std::vector<std::vector<std::pair<int32_t, double>>>& rows) {
    HostCSR c;
    c.nrows = nrows;
    c.ncols = ncols;
    c.rowptr.assign(nrows + 1, 0);
    for (int64_t r = 0; r < nrows; ++r) {
        auto& v = rows[r];
        std::sort(v.begin(), v.end(), [](auto& a, auto& b) { return a.first < b.first; });
        int32_t last = -1;
        for (auto& e : v) {
            if (e.first == last) {
                c.val.back() += e.second;
            } else {
                c.col.push_back(e.first);
                c.val.push_back(e.second);
                last = e.first;
            }
        }
        c.rowptr[r + 1] = (int32_t)c.col.size();
    }
    return c;
}

HostCSR transpose(const HostCSR& a) {
    std::vector<std::vector<std::pair<int32_t, double>>> rows(a.ncols);
    for (int64_t r = 0; r < a.nrows; ++r)
        for (int32_t p = a.rowptr[r]; p < a.rowptr[r + 1]; ++p) rows[a.col[p]].push_back({(int32_t)r, a.val[p]});
    return triplets_to_csr(a.ncols, a.nrows, rows);
}

bool invert_dense(std::vector<double>& a, int n) {
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        if (std::fabs(a[(size_t)piv * n + c]) < 1e-300) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        double d = 1.0 / a[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= d;
            inv[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    a.swap(inv);
    return true;
}

// Vertex numbering of one level of the nested P1 grids, and its fixed vertex
// (the pinned pressure, when there is one).  The level operator itself is
// filled by schur_values().
void build_level(const mhd_mesh_desc* d, int level, HostLevel& L, std::vector<uint8_t>& fixed,
                 std::vector<int32_t>& vid) {
    Grid g = make_grid(d, level);
    L.nx = g.nx;
    L.ny = g.ny;
    L.h = g.h;
    int nv = 0;
    vid = vertex_ids(g, nv);
    L.n = nv;
    fixed.assign(nv, 0);
    if (!(d->kind == MHD_MESH_STEP_CHANNEL && d->natural_outflow))
        fixed[0] = 1;   // pinned pressure: first vertex in row-major order
}

// C = A diag(w) B (w empty: identity); the pattern is the symbolic product
// (entries are kept even when their value is zero, so the pattern does not
// depend on the values).
HostCSR spgemm(const HostCSR& A, const std::vector<double>& w, const HostCSR& B) {
    HostCSR C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.rowptr.assign(A.nrows + 1, 0);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> mark(B.ncols, -1), cols;
    for (int64_t r = 0; r < A.nrows; ++r) {
        cols.clear();
        for (int32_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
            int32_t k = A.col[p];
            double a = A.val[p] * (w.empty() ? 1.0 : w[k]);
            for (int32_t q = B.rowptr[k]; q < B.rowptr[k + 1]; ++q) {
                int32_t c = B.col[q];
                if (mark[c] != (int32_t)r) {
                    mark[c] = (int32_t)r;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += a * B.val[q];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            C.col.push_back(c);
            C.val.push_back(acc[c]);
        }
        C.rowptr[r + 1] = (int32_t)C.col.size();
    }
    return C;
}

// identity row and column for a fixed node (the row is replaced by its
// diagonal entry; column entries of other rows are kept as explicit zeros)
void fix_node(HostCSR& A, int32_t f) {
    HostCSR B;
    B.nrows = A.nrows;
    B.ncols = A.ncols;
    B.rowptr.assign(A.nrows + 1, 0);
    for (int64_t r = 0; r < A.nrows; ++r) {
        if (r == f) {
            B.col.push_back(f);
            B.val.push_back(1.0);
        } else {
            for (int32_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
                B.col.push_back(A.col[p]);
                B.val.push_back(A.col[p] == f ? 0.0 : A.val[p]);
            }
        }
        B.rowptr[r + 1] = (int32_t)B.col.size();
    }
    A = std::move(B);
}

// alpha A + beta B on the union pattern (entries of either kept)
HostCSR add_csr(const HostCSR& A, double alpha, const HostCSR& B, double beta) {
    HostCSR C;
    C.nrows = A.nrows;
    C.ncols = A.ncols;
    C.rowptr.assign(A.nrows + 1, 0);
    for (int64_t r = 0; r < A.nrows; ++r) {
        int32_t p = A.rowptr[r], q = B.rowptr[r];
        const int32_t pe = A.rowptr[r + 1], qe = B.rowptr[r + 1];
        while (p < pe || q < qe) {
            const int32_t ca = p < pe ? A.col[p] : INT32_MAX, cb = q < qe ? B.col[q] : INT32_MAX;
            const int32_t c = std::min(ca, cb);
            double v = 0.0;
            if (ca == c) v += alpha * A.val[p++];
            if (cb == c) v += beta * B.val[q++];
            C.col.push_back(c);
            C.val.push_back(v);
        }
        C.rowptr[r + 1] = (int32_t)C.col.size();
    }
    return C;
}

HostCSR diag_csr(const std::vector<double>& d) {
    HostCSR C;
    C.nrows = C.ncols = (int64_t)d.size();
    C.rowptr.resize(d.size() + 1);
    for (size_t i = 0; i < d.size(); ++i) {
        C.rowptr[i] = (int32_t)i;
        C.col.push_back((int32_t)i);
        C.val.push_back(d[i]);
    }
    C.rowptr[d.size()] = (int32_t)d.size();
    return C;
}

// [A | B] with the columns of B numbered after those of A
HostCSR hcat_csr(const HostCSR& A, const HostCSR& B) {
    HostCSR C;
    C.nrows = A.nrows;
    C.ncols = A.ncols + B.ncols;
    C.rowptr.assign(A.nrows + 1, 0);
    for (int64_t r = 0; r < A.nrows; ++r) {
        for (int32_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
            C.col.push_back(A.col[p]);
            C.val.push_back(A.val[p]);
        }
        for (int32_t p = B.rowptr[r]; p < B.rowptr[r + 1]; ++p) {
            C.col.push_back((int32_t)(A.ncols + B.col[p]));
            C.val.push_back(B.val[p]);
        }
        C.rowptr[r + 1] = (int32_t)C.col.size();
    }
    return C;
}

// Two fused steps of a level's V(2,2)-cycle with damped Jacobi smoothing
// (E = I - w D^-1 L), each a single sparse operator on stacked inputs:
//   down:  bc = R b - (R L) x2           = [R | -R L] [b; x2]
//          (the residual of the pre-smoothed x2, restricted);
//   up:    x = E x2 + (E P) xc + w D^-1 b = [E | E P | w D^-1] [x2; xc; b]
//          (the coarse correction prolonged into x2, then one smoothing sweep).
// Patterns are symbolic products, so they depend only on the hierarchy.
void fused_level_ops(HostLevel& F, double w) {
    std::vector<double> ones(F.n, 1.0), wd(F.dinv);
    for (double& v : wd) v *= w;
    const HostCSR I = diag_csr(ones);
    const HostCSR RL = spgemm(F.R, {}, F.L);
    F.Dn = hcat_csr(F.R, add_csr(RL, -1.0, RL, 0.0));
    const HostCSR DL = spgemm(diag_csr(F.dinv), {}, F.L);
    const HostCSR E = add_csr(I, 1.0, DL, -w);
    F.Up = hcat_csr(hcat_csr(E, spgemm(E, {}, F.P)), diag_csr(wd));
}

}  // namespace

// Pressure Schur-complement approximation S_hat = B D^{-1} B^T with
// D = diag(M)/dt + nu_c diag(K) (the diagonal of the velocity block without its
// convection part, whose skew-symmetric form has a zero diagonal), and its
// Galerkin multigrid hierarchy S_{l+1} = P_l^T S_l P_l over the nested P1
// grids.  Values are recomputed when (dt, nu_c) change; patterns never do.
mhd_status schur_values(HostMesh& m, double dt, double nu_c) {
    const int nP2 = m.nP2;
    std::vector<double> dinv_u(2 * (size_t)nP2, 0.0);
    for (int i = 0; i < nP2; ++i) {
        double d = m.diagM[i] / dt + nu_c * m.diagK[i];
        dinv_u[2 * i] = dinv_u[2 * i + 1] = (d > 0) ? 1.0 / d : 0.0;
    }
    std::vector<HostLevel>& L = m.levels;
    HostCSR S0 = spgemm(m.Bs, dinv_u, m.Bts);
    if (m.pin >= 0) fix_node(S0, m.pin);
    for (size_t l = 0; l < L.size(); ++l) {
        HostCSR cur;
        if (l == 0) {
            cur = std::move(S0);
        } else {
            HostCSR T = spgemm(L[l - 1].L, {}, L[l - 1].P);
            cur = spgemm(L[l - 1].R, {}, T);
            if (m.pin >= 0) fix_node(cur, 0);
        }
        if (!L[l].L.col.empty() && (L[l].L.col.size() != cur.col.size())) {
            set_error("schur hierarchy: pattern changed");
            return MHD_EINVAL;
        }
        L[l].L = std::move(cur);
        L[l].dinv.assign(L[l].n, 0.0);
        for (int v = 0; v < L[l].n; ++v)
            for (int32_t p = L[l].L.rowptr[v]; p < L[l].L.rowptr[v + 1]; ++p)
                if (L[l].L.col[p] == v) L[l].dinv[v] = L[l].L.val[p] != 0.0 ? 1.0 / L[l].L.val[p] : 0.0;
    }
    // The discontinuous pressure levels of Scott-Vogelius meshes have a larger
    // spectrum of D^-1 L than the vertex grids (about 3.9 and 3.5 against 2),
    // where the damping 0.8 would amplify the oscillating modes: damp them by
    // 1.9 / lambda_max, lambda_max estimated by power iteration (deterministic start)
    for (size_t l = 0; l + 1 < L.size(); ++l) {
        HostLevel& F = L[l];
        if (!F.dg) continue;
        std::vector<double> v(F.n), w(F.n);
        for (int i = 0; i < F.n; ++i) v[i] = ((i & 1) ? -1.0 : 1.0) * (1.0 + 0.01 * (i % 13));
        double lam = 0.0;
        for (int it = 0; it < 60; ++it) {
            double nv = 0.0, nw = 0.0;
            for (int r = 0; r < F.n; ++r) {
                double acc = 0.0;
                for (int32_t p = F.L.rowptr[r]; p < F.L.rowptr[r + 1]; ++p) acc += F.L.val[p] * v[F.L.col[p]];
                w[r] = F.dinv[r] * acc;
                nv += v[r] * v[r];
                nw += w[r] * w[r];
            }
            lam = std::sqrt(nw / nv);
            const double inv = 1.0 / std::sqrt(nw);
            for (int r = 0; r < F.n; ++r) v[r] = w[r] * inv;
        }
        F.omega = std::min(kMgOmega, 1.9 / lam);
    }
    for (size_t l = 0; l + 1 < L.size(); ++l) {
        const int64_t nd = L[l].Dn.nnz(), nu = L[l].Up.nnz();
        fused_level_ops(L[l], L[l].omega);
        if ((nd && nd != L[l].Dn.nnz()) || (nu && nu != L[l].Up.nnz())) {
            set_error("schur hierarchy: fused pattern changed");
            return MHD_EINVAL;
        }
    }
    HostLevel& Lc = L.back();
    Lc.cinv.assign((size_t)Lc.n * Lc.n, 0.0);
    for (int r = 0; r < Lc.n; ++r)
        for (int32_t p = Lc.L.rowptr[r]; p < Lc.L.rowptr[r + 1]; ++p) Lc.cinv[(size_t)r * Lc.n + Lc.L.col[p]] = Lc.L.val[p];
    if (!invert_dense(Lc.cinv, Lc.n)) {
        // degenerate meshes (a single cell) give a singular approximation: fall
        // back to its diagonal inverse, which still defines a preconditioner
        Lc.cinv.assign((size_t)Lc.n * Lc.n, 0.0);
        for (int r = 0; r < Lc.n; ++r) Lc.cinv[(size_t)r * Lc.n + r] = Lc.dinv[r];
    }
    m.schur_dt = dt;
    m.schur_nuc = nu_c;
    return MHD_OK;
}

// ---------------------------------------------------------------- reference tables
void make_ref_tables(RefTables& t) { t = build_ref_tables(); }

// ---------------------------------------------------------------- mesh
// Barycentric (Alfeld) refinement of the cell triangulation, the meshes on
// which Section 2 places the Scott-Vogelius pair: each triangle (p0, p1, p2)
// of a cell (lower (v00, v10, v11), then upper (v00, v11, v01)) with
// barycentre g becomes (p0, p1, g), (p1, p2, g), (p2, p0, g), in that order.
// Every P2 node of the refined mesh lies on the grid of sixth steps (h/6);
// nodes are numbered row-major on that grid (y slowest).  The pressure is
// discontinuous P1: unknown 3 e + k belongs to vertex k of element e.
void alfeld_nodes(const Grid& g, const mhd_mesh_desc* d, HostMesh& m) {
    const int64_t NX = 6 * (int64_t)g.nx + 1;
    std::vector<int64_t> key;   // 6 node keys K * NX + I per element
    for (int k = 0; k < g.ny; ++k)
        for (int i = 0; i < g.nx; ++i) {
            if (!g.cell(i, k)) continue;
            const int64_t X = 6 * (int64_t)i, Y = 6 * (int64_t)k;
            const int64_t mac[2][3][2] = {{{X, Y}, {X + 6, Y}, {X + 6, Y + 6}}, {{X, Y}, {X + 6, Y + 6}, {X, Y + 6}}};
            for (const auto& t : mac) {
                const int64_t gx = (t[0][0] + t[1][0] + t[2][0]) / 3, gy = (t[0][1] + t[1][1] + t[2][1]) / 3;
                for (int s = 0; s < 3; ++s) {
                    const int64_t ax = t[s][0], ay = t[s][1], bx = t[(s + 1) % 3][0], by = t[(s + 1) % 3][1];
                    const int64_t pts[6][2] = {{ax, ay}, {bx, by}, {gx, gy}, {(ax + bx) / 2, (ay + by) / 2},
                                               {(bx + gx) / 2, (by + gy) / 2}, {(gx + ax) / 2, (gy + ay) / 2}};
                    for (const auto& q : pts) key.push_back(q[1] * NX + q[0]);
                }
            }
        }
    std::vector<int64_t> nodes(key);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    const int nP2 = (int)nodes.size(), n_el = (int)(key.size() / 6);
    m.nP2 = nP2;
    m.n_el = n_el;
    m.nP1 = 3 * n_el;
    m.tri.resize(key.size());
    for (size_t c = 0; c < key.size(); ++c)
        m.tri[c] = (int32_t)(std::lower_bound(nodes.begin(), nodes.end(), key[c]) - nodes.begin());
    m.tri1.resize((size_t)3 * n_el);
    for (int c = 0; c < 3 * n_el; ++c) m.tri1[c] = c;
    m.xy.assign((size_t)nP2 * 2, 0.0);
    for (int id = 0; id < nP2; ++id) {
        m.xy[2 * id] = g.x0 + (double)(nodes[id] % NX) * g.h / 6.0;
        m.xy[2 * id + 1] = g.y0 + (double)(nodes[id] / NX) * g.h / 6.0;
    }
    // boundary: nodes of the element edges that belong to one element only
    std::vector<std::pair<int64_t, int32_t>> edges;   // (vertex pair, midpoint)
    for (int e = 0; e < n_el; ++e) {
        const int32_t* t = &m.tri[(size_t)e * 6];
        for (int s = 0; s < 3; ++s) {
            const int32_t a = t[s], b = t[(s + 1) % 3];
            edges.push_back({(int64_t)std::min(a, b) * nP2 + std::max(a, b), t[3 + s]});
        }
    }
    std::sort(edges.begin(), edges.end());
    m.bnd.assign(nP2, 0);
    for (size_t c = 0; c < edges.size();) {
        size_t r = c;
        while (r < edges.size() && edges[r].first == edges[c].first) ++r;
        if (r - c == 1) {
            m.bnd[edges[c].first / nP2] = m.bnd[edges[c].first % nP2] = m.bnd[edges[c].second] = 1;
        }
        c = r;
    }
    m.dir.assign(nP2, 0);
    m.p1_of_p2.assign(nP2, -1);
    for (int id = 0; id < nP2; ++id) {
        const bool outflow = d->natural_outflow && std::fabs(m.xy[2 * id] - m.xmax) < 1e-9 * (1 + m.xmax);
        m.dir[id] = (m.bnd[id] && !outflow) ? 1 : 0;
    }
    m.dir_nodes.clear();
    for (int i = 0; i < nP2; ++i)
        if (m.dir[i]) m.dir_nodes.push_back(i);
    m.hs_p2.clear();
    m.cell_el.clear();
}

mhd_status build_mesh(const mhd_mesh_desc* d, HostMesh& m, bool full) {
    if (!d) {
        set_error("mhd_ens_mesh: null descriptor");
        return MHD_EINVAL;
    }
    if (d->kind != MHD_MESH_UNIT_SQUARE && d->kind != MHD_MESH_STEP_CHANNEL) {
        set_error("mhd_ens_mesh: unknown mesh kind");
        return MHD_EINVAL;
    }
    if (d->nx < 1 || d->nx > 4096) {
        set_error("mhd_ens_mesh: nx must be in [1, 4096]");
        return MHD_EINVAL;
    }
    if (d->element != MHD_ELEMENT_TAYLOR_HOOD && d->element != MHD_ELEMENT_SCOTT_VOGELIUS) {
        set_error("mhd_ens_mesh: element must be MHD_ELEMENT_TAYLOR_HOOD or MHD_ELEMENT_SCOTT_VOGELIUS");
        return MHD_EINVAL;
    }
    if (d->kind == MHD_MESH_UNIT_SQUARE && d->natural_outflow) {
        set_error("mhd_ens_mesh: natural outflow is only defined for the step channel");
        return MHD_EINVAL;
    }
    m.desc = *d;
    Grid g = make_grid(d, 0);
    m.nx = g.nx;
    m.ny = g.ny;
    m.h = g.h;
    m.x0 = g.x0;
    m.y0 = g.y0;
    m.xmax = g.x0 + g.nx * g.h;
    const int NX = 2 * g.nx + 1, NY = 2 * g.ny + 1;
    // ---- P2 nodes on the half-step grid
    std::vector<int32_t> pid((size_t)NX * NY, -1);
    std::vector<uint8_t> pbnd((size_t)NX * NY, 0);
    int nP2 = 0;
    for (int K = 0; K < NY; ++K)
        for (int I = 0; I < NX; ++I) {
            int cnt = 0, tot = 0;
            if ((I & 1) == 0 && (K & 1) == 0) {
                cnt = g.vertex_cells(I / 2, K / 2);
                tot = 4;
            } else if ((I & 1) == 1 && (K & 1) == 0) {
                int i = (I - 1) / 2, k = K / 2;
                cnt = (int)g.cell(i, k - 1) + (int)g.cell(i, k);
                tot = 2;
            } else if ((I & 1) == 0 && (K & 1) == 1) {
                int i = I / 2, k = (K - 1) / 2;
                cnt = (int)g.cell(i - 1, k) + (int)g.cell(i, k);
                tot = 2;
            } else {
                cnt = (int)g.cell((I - 1) / 2, (K - 1) / 2);
                tot = 1;
            }
            if (cnt > 0) {
                pid[(size_t)K * NX + I] = nP2++;
                pbnd[(size_t)K * NX + I] = (cnt < tot) ? 1 : 0;
            }
        }
    m.nP2 = nP2;
    int nP1 = 0;
    std::vector<int32_t> vid = vertex_ids(g, nP1);
    m.nP1 = nP1;
    int n_el = 0;
    for (int k = 0; k < g.ny; ++k)
        for (int i = 0; i < g.nx; ++i) n_el += g.cell(i, k) ? 2 : 0;
    m.n_el = n_el;
    const bool sv = d->element == MHD_ELEMENT_SCOTT_VOGELIUS;
    if (sv) {   // each triangle adds its barycentre and three inner edge midpoints
        m.nP2 = nP2 + 4 * n_el;
        m.n_el = 3 * n_el;
        m.nP1 = 3 * m.n_el;
    }
    if (!full) return MHD_OK;
    int e = 0;
    if (sv) {
        alfeld_nodes(g, d, m);
        nP2 = m.nP2;
        nP1 = m.nP1;
        n_el = m.n_el;
    } else {
    m.xy.assign((size_t)nP2 * 2, 0.0);
    m.bnd.assign(nP2, 0);
    m.dir.assign(nP2, 0);
    m.p1_of_p2.assign(nP2, -1);
    for (int K = 0; K < NY; ++K)
        for (int I = 0; I < NX; ++I) {
            int id = pid[(size_t)K * NX + I];
            if (id < 0) continue;
            double x = g.x0 + I * 0.5 * g.h, y = g.y0 + K * 0.5 * g.h;
            m.xy[2 * id] = x;
            m.xy[2 * id + 1] = y;
            m.bnd[id] = pbnd[(size_t)K * NX + I];
            bool outflow = d->natural_outflow && std::fabs(x - m.xmax) < 1e-9 * (1 + m.xmax);
            m.dir[id] = (m.bnd[id] && !outflow) ? 1 : 0;
            if ((I & 1) == 0 && (K & 1) == 0) m.p1_of_p2[id] = vid[(size_t)(K / 2) * (g.nx + 1) + I / 2];
        }
    m.dir_nodes.clear();
    for (int i = 0; i < nP2; ++i)
        if (m.dir[i]) m.dir_nodes.push_back(i);
    // ---- elements
    m.tri.resize((size_t)n_el * 6);
    m.tri1.resize((size_t)n_el * 3);
    m.hs_p2 = pid;
    m.cell_el.assign((size_t)g.nx * g.ny, -1);
    auto P = [&](int I, int K) { return pid[(size_t)K * NX + I]; };
    auto V = [&](int i, int k) { return vid[(size_t)k * (g.nx + 1) + i]; };
    for (int k = 0; k < g.ny; ++k)
        for (int i = 0; i < g.nx; ++i) {
            if (!g.cell(i, k)) continue;
            int I = 2 * i, K = 2 * k;
            m.cell_el[(size_t)k * g.nx + i] = e;
            // lower (v00, v10, v11), upper (v00, v11, v01); locals 3,4,5 = mid(0,1), mid(1,2), mid(2,0)
            int lo[6] = {P(I, K), P(I + 2, K), P(I + 2, K + 2), P(I + 1, K), P(I + 2, K + 1), P(I + 1, K + 1)};
            int up[6] = {P(I, K), P(I + 2, K + 2), P(I, K + 2), P(I + 1, K + 1), P(I + 1, K + 2), P(I, K + 1)};
            int lo1[3] = {V(i, k), V(i + 1, k), V(i + 1, k + 1)};
            int up1[3] = {V(i, k), V(i + 1, k + 1), V(i, k + 1)};
            for (int a = 0; a < 6; ++a) m.tri[(size_t)e * 6 + a] = lo[a];
            for (int a = 0; a < 3; ++a) m.tri1[(size_t)e * 3 + a] = lo1[a];
            ++e;
            for (int a = 0; a < 6; ++a) m.tri[(size_t)e * 6 + a] = up[a];
            for (int a = 0; a < 3; ++a) m.tri1[(size_t)e * 3 + a] = up1[a];
            ++e;
        }
    }
    // ---- patterns
    {
        std::vector<std::vector<int32_t>> rA(nP2), rBt(nP2), rB(nP1);
        for (e = 0; e < n_el; ++e) {
            const int32_t* t = &m.tri[(size_t)e * 6];
            const int32_t* t1 = &m.tri1[(size_t)e * 3];
            for (int a = 0; a < 6; ++a) {
                for (int b = 0; b < 6; ++b) rA[t[a]].push_back(t[b]);
                for (int k = 0; k < 3; ++k) {
                    rBt[t[a]].push_back(t1[k]);
                    rB[t1[k]].push_back(t[a]);
                }
            }
        }
        auto finish = [](std::vector<std::vector<int32_t>>& rows, int64_t ncols, HostCSR& c) {
            c.nrows = (int64_t)rows.size();
            c.ncols = ncols;
            c.rowptr.assign(rows.size() + 1, 0);
            c.col.clear();
            for (size_t r = 0; r < rows.size(); ++r) {
                auto& v = rows[r];
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end()), v.end());
                c.col.insert(c.col.end(), v.begin(), v.end());
                c.rowptr[r + 1] = (int32_t)c.col.size();
                std::vector<int32_t>().swap(v);
            }
        };
        finish(rA, nP2, m.A);
        finish(rBt, nP1, m.Bt);
        finish(rB, nP2, m.B);
    }
    auto slot = [](const HostCSR& c, int32_t r, int32_t col) {
        const int32_t* b = c.col.data() + c.rowptr[r];
        const int32_t* en = c.col.data() + c.rowptr[r + 1];
        const int32_t* p = std::lower_bound(b, en, col);
        return (int32_t)(p - c.col.data());
    };
    m.slotA.resize((size_t)n_el * 36);
    std::vector<int32_t> slotB((size_t)n_el * 18), slotBt((size_t)n_el * 18);
    for (e = 0; e < n_el; ++e) {
        const int32_t* t = &m.tri[(size_t)e * 6];
        const int32_t* t1 = &m.tri1[(size_t)e * 3];
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) m.slotA[(size_t)e * 36 + a * 6 + b] = slot(m.A, t[a], t[b]);
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 6; ++a) {
                slotB[(size_t)e * 18 + k * 6 + a] = slot(m.B, t1[k], t[a]);
                slotBt[(size_t)e * 18 + k * 6 + a] = slot(m.Bt, t[a], t1[k]);
            }
    }
    auto gather = [](const std::vector<int32_t>& slots, int64_t nslots, std::vector<int32_t>& ptr,
                     std::vector<int32_t>& idx) {
        ptr.assign(nslots + 1, 0);
        for (int32_t s : slots) ptr[s + 1]++;
        for (int64_t i = 0; i < nslots; ++i) ptr[i + 1] += ptr[i];
        idx.assign(slots.size(), 0);
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (size_t c = 0; c < slots.size(); ++c) idx[fill[slots[c]]++] = (int32_t)c;
    };
    // transposition maps: A slot (i,k) -> slot (k,i); B^T slot (i,m) -> B slot (m,i)
    m.permA.resize(m.A.nnz());
    for (int i = 0; i < nP2; ++i)
        for (int32_t p = m.A.rowptr[i]; p < m.A.rowptr[i + 1]; ++p) m.permA[p] = slot(m.A, m.A.col[p], i);
    m.permBtB.resize(m.Bt.nnz());
    for (int i = 0; i < nP2; ++i)
        for (int32_t p = m.Bt.rowptr[i]; p < m.Bt.rowptr[i + 1]; ++p) m.permBtB[p] = slot(m.B, m.Bt.col[p], i);
    gather(m.slotA, m.A.nnz(), m.gA_ptr, m.gA_idx);
    gather(slotB, m.B.nnz(), m.gB_ptr, m.gB_idx);
    gather(slotBt, m.Bt.nnz(), m.gBt_ptr, m.gBt_idx);
    // ---- node -> (element, local) incidence
    m.inc_ptr.assign(nP2 + 1, 0);
    for (e = 0; e < n_el; ++e)
        for (int a = 0; a < 6; ++a) m.inc_ptr[m.tri[(size_t)e * 6 + a] + 1]++;
    for (int i = 0; i < nP2; ++i) m.inc_ptr[i + 1] += m.inc_ptr[i];
    m.inc.assign(m.inc_ptr[nP2], 0);
    {
        std::vector<int32_t> fill(m.inc_ptr.begin(), m.inc_ptr.end() - 1);
        for (e = 0; e < n_el; ++e)
            for (int a = 0; a < 6; ++a) m.inc[fill[m.tri[(size_t)e * 6 + a]]++] = e * 8 + a;
    }
    // ---- lumped P1 mass
    m.mp.assign(nP1, 0.0);
    for (e = 0; e < n_el; ++e) {
        const int32_t* t = &m.tri[(size_t)e * 6];
        double gl[3][2], area;
        grad_bary(&m.xy[2 * t[0]], &m.xy[2 * t[1]], &m.xy[2 * t[2]], gl, area);
        for (int k = 0; k < 3; ++k) m.mp[m.tri1[(size_t)e * 3 + k]] += area / 3.0;
    }
    // ---- pressure fixing and multigrid hierarchy
    m.levels.clear();
    std::vector<std::vector<uint8_t>> fixed;
    std::vector<std::vector<int32_t>> vids;
    const bool pinned = !(d->kind == MHD_MESH_STEP_CHANNEL && d->natural_outflow);
    // Scott-Vogelius: the finest levels are discontinuous pressure spaces, on the
    // refinement (level 0, the pressure space itself) and on the unrefined mesh
    // (level 1: linear on each unrefined triangle, 3 unknowns each); the levels
    // below are the vertex grids of the unrefined mesh and their coarsenings
    int off = 0;
    if (sv) {
        for (int q = 0; q < 2; ++q) {
            if (q == 1 && m.levels.back().n <= kCoarseMax) break;
            HostLevel Ld;
            Ld.nx = g.nx;
            Ld.ny = g.ny;
            Ld.h = g.h;
            Ld.n = q == 0 ? nP1 : nP1 / 3;
            Ld.dg = true;
            m.levels.push_back(std::move(Ld));
            fixed.push_back(std::vector<uint8_t>(m.levels.back().n, 0));
            if (pinned) fixed.back()[0] = 1;
            vids.push_back({});
            ++off;
        }
    }
    int level = 0;
    while (!sv || m.levels.back().n > kCoarseMax) {
        HostLevel L;
        std::vector<uint8_t> fx;
        std::vector<int32_t> vi;
        build_level(d, level, L, fx, vi);
        m.levels.push_back(std::move(L));
        fixed.push_back(std::move(fx));
        vids.push_back(std::move(vi));
        const HostLevel& cur = m.levels.back();
        bool can_halve;
        if (d->kind == MHD_MESH_UNIT_SQUARE)
            can_halve = (cur.nx % 2 == 0) && cur.nx >= 4;
        else
            can_halve = ((d->nx >> level) % 2 == 0);
        if (cur.n <= kCoarseMax || !can_halve) break;
        ++level;
    }
    if (m.levels.back().n > kCoarseDenseMax) {
        set_error("mhd_ens_mesh: the pressure multigrid cannot coarsen this mesh to a level of at most " +
                  std::to_string(kCoarseDenseMax) + " vertices for its dense coarse solve (coarsest level: " +
                  std::to_string(m.levels.back().n) + " vertices); nx needs more factors of two");
        return MHD_EINVAL;
    }
    m.pfix = fixed[0];
    m.pin = pinned ? 0 : -1;
    // Scott-Vogelius transfers, exact for functions linear on each unrefined triangle:
    //   level 1 -> 0: an element vertex takes the value at that vertex of the unrefined
    //     triangle (1 at its vertices, 1/3 of each at the barycentre);
    //   vertex grid -> level 1: each unrefined triangle takes its vertex values.
    // Element e = 3 E + s of the refinement is (p_s, p_{s+1}, g) in unrefined triangle E.
    if (sv && m.levels.size() > 1) {
        HostLevel& F = m.levels[0];
        std::vector<std::vector<std::pair<int32_t, double>>> rows(F.n);
        for (e = 0; e < n_el; ++e) {
            const int E = e / 3, sub = e % 3;
            for (int k = 0; k < 3; ++k) {
                const int32_t f = m.tri1[(size_t)e * 3 + k];
                if (fixed[0][f]) continue;
                std::vector<std::pair<int32_t, double>> ent;
                if (k < 2)
                    ent.push_back({3 * E + (sub + k) % 3, 1.0});
                else
                    for (int q = 0; q < 3; ++q) ent.push_back({3 * E + q, 1.0 / 3.0});
                for (auto& en : ent)
                    if (!fixed[1][en.first]) rows[f].push_back(en);
            }
        }
        F.P = triplets_to_csr(F.n, m.levels[1].n, rows);
        F.R = transpose(F.P);
    }
    if (sv && m.levels.size() > 2) {
        HostLevel& F = m.levels[1];
        const HostLevel& C = m.levels[2];
        std::vector<std::vector<std::pair<int32_t, double>>> rows(F.n);
        for (int f = 0; f < F.n; ++f) {
            if (fixed[1][f]) continue;
            const int32_t node = m.tri[(size_t)f * 6];   // vertex 0 of element f = vertex f % 3 of triangle f / 3
            const int64_t ci = std::llround((m.xy[2 * node] - g.x0) / g.h);
            const int64_t ck = std::llround((m.xy[2 * node + 1] - g.y0) / g.h);
            const int32_t c = vids[2][(size_t)ck * (C.nx + 1) + ci];
            if (c >= 0 && !fixed[2][c]) rows[f].push_back({c, 1.0});
        }
        F.P = triplets_to_csr(F.n, C.n, rows);
        F.R = transpose(F.P);
    }
    // interpolation from level l+1 to level l: P1 interpolation on the coarse triangulation
    for (size_t l = off; l + 1 < m.levels.size(); ++l) {
        HostLevel& F = m.levels[l];
        const HostLevel& C = m.levels[l + 1];
        std::vector<std::vector<std::pair<int32_t, double>>> rows(F.n);
        auto cid = [&](int ci, int ck) -> int32_t {
            if (ci < 0 || ck < 0 || ci > C.nx || ck > C.ny) return -1;
            return vids[l + 1][(size_t)ck * (C.nx + 1) + ci];
        };
        for (int k = 0; k <= F.ny; ++k)
            for (int i = 0; i <= F.nx; ++i) {
                int f = vids[l][(size_t)k * (F.nx + 1) + i];
                if (f < 0 || fixed[l][f]) continue;
                std::vector<std::pair<int32_t, double>> ent;
                if (i % 2 == 0 && k % 2 == 0) {
                    ent.push_back({cid(i / 2, k / 2), 1.0});
                } else if (i % 2 == 1 && k % 2 == 0) {
                    ent.push_back({cid((i - 1) / 2, k / 2), 0.5});
                    ent.push_back({cid((i + 1) / 2, k / 2), 0.5});
                } else if (i % 2 == 0 && k % 2 == 1) {
                    ent.push_back({cid(i / 2, (k - 1) / 2), 0.5});
                    ent.push_back({cid(i / 2, (k + 1) / 2), 0.5});
                } else {
                    ent.push_back({cid((i - 1) / 2, (k - 1) / 2), 0.5});
                    ent.push_back({cid((i + 1) / 2, (k + 1) / 2), 0.5});
                }
                for (auto& en : ent)
                    if (en.first >= 0 && !fixed[l + 1][en.first]) rows[f].push_back(en);
            }
        F.P = triplets_to_csr(F.n, C.n, rows);
        F.R = transpose(F.P);
    }
    // ---- host copies of the divergence operator and of diag(M), diag(K) (for the Schur approximation)
    {
        RefTables t;
        make_ref_tables(t);
        std::vector<double> eb((size_t)n_el * 36);
        m.diagM.assign(nP2, 0.0);
        m.diagK.assign(nP2, 0.0);
        for (e = 0; e < n_el; ++e) {
            const int32_t* tr = &m.tri[(size_t)e * 6];
            const double* p0 = &m.xy[2 * tr[0]];
            const double* p1 = &m.xy[2 * tr[1]];
            const double* p2 = &m.xy[2 * tr[2]];
            double a = p1[0] - p0[0], b = p2[0] - p0[0], c = p1[1] - p0[1], dd = p2[1] - p0[1];
            double det = a * dd - b * c;
            double Ji[2][2] = {{dd / det, -b / det}, {-c / det, a / det}};
            double G[2][2];
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y) G[x][y] = Ji[x][0] * Ji[y][0] + Ji[x][1] * Ji[y][1];
            for (int aa = 0; aa < 6; ++aa) {
                m.diagM[tr[aa]] += det * t.Mhat[aa][aa];
                double k = 0.0;
                for (int x = 0; x < 2; ++x)
                    for (int y = 0; y < 2; ++y) k += t.Khat[aa][aa][x][y] * G[x][y];
                m.diagK[tr[aa]] += det * k;
            }
            for (int k = 0; k < 3; ++k)
                for (int aa = 0; aa < 6; ++aa)
                    for (int dir = 0; dir < 2; ++dir) {
                        double v = 0.0;
                        for (int x = 0; x < 2; ++x) v += t.Bhat[k][aa][x] * Ji[x][dir];
                        eb[(size_t)e * 36 + (k * 6 + aa) * 2 + dir] = det * v;
                    }
        }
        // scalar CSRs over velocity unknowns 2i+c: Bs (P1 x 2 nP2), Bts (2 nP2 x P1)
        std::vector<std::vector<std::pair<int32_t, double>>> rb(nP1), rbt(2 * (size_t)nP2);
        for (int k = 0; k < nP1; ++k) {
            if (k == m.pin) continue;                    // pinned row of B is zero
            for (int32_t p = m.B.rowptr[k]; p < m.B.rowptr[k + 1]; ++p) {
                double v[2] = {0.0, 0.0};
                for (int32_t q = m.gB_ptr[p]; q < m.gB_ptr[p + 1]; ++q)
                    for (int dir = 0; dir < 2; ++dir) v[dir] += eb[(size_t)m.gB_idx[q] * 2 + dir];
                for (int dir = 0; dir < 2; ++dir) {
                    rb[k].push_back({2 * m.B.col[p] + dir, v[dir]});
                    if (!m.dir[m.B.col[p]]) rbt[2 * (size_t)m.B.col[p] + dir].push_back({k, v[dir]});
                }
            }
        }
        m.Bs = triplets_to_csr(nP1, 2 * (int64_t)nP2, rb);
        m.Bts = triplets_to_csr(2 * (int64_t)nP2, nP1, rbt);
    }
    return schur_values(m, 1.0, 0.0);
}

void mesh_counts(const HostMesh& m, mhd_mesh_info* info) {
    info->n_el = m.n_el;
    info->nP2 = m.nP2;
    info->nP1 = m.nP1;
    info->n_u = 2 * (int64_t)m.nP2;
    info->n = 2 * (int64_t)m.nP2 + m.nP1;
    info->nnz_A = m.A.nnz();
    info->nnz_B = m.B.nnz();
    info->nnz = 2 * m.A.nnz() + 2 * m.Bt.nnz() + 2 * m.B.nnz() + (m.pin >= 0 ? 1 : 0);
    int64_t nb = 0;
    for (auto b : m.bnd) nb += b;
    info->n_bd = nb;
    info->n_dir = (int64_t)m.dir_nodes.size();
    info->pin = m.pin;
    info->mg_levels = (int32_t)m.levels.size();
}

}  // namespace mhd
