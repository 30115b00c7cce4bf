// Internal definitions of libmhd_ens: host mesh structures, device mirrors,
// launcher prototypes.  Not part of the public ABI (include/mhd_ens.h is).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mhd_ens.h"

namespace mhd {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
std::string hip_error_string(int code);

// ------------------------------------------------------------------ host CSR
struct HostCSR {
    int64_t nrows = 0, ncols = 0;
    std::vector<int32_t> rowptr, col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

// One level of the pressure multigrid hierarchy (P1 Laplacian of the level's
// triangulation, its inverse diagonal, interpolation from the next coarser
// level and its transpose).
constexpr double kMgOmega = 0.8;   // Jacobi damping of the pressure multigrid
struct HostLevel {
    double omega = kMgOmega;     // Jacobi damping of this level's sweeps
    bool dg = false;             // a discontinuous pressure level (Scott-Vogelius)
    int nx = 0, ny = 0;          // cells of this level
    double h = 0;
    int n = 0;                   // active vertices
    HostCSR L;                   // stiffness with fixed rows replaced by identity
    std::vector<double> dinv;    // 1 / diag(L)
    HostCSR P;                   // (n x n_coarse) interpolation from level+1 (empty on coarsest)
    HostCSR R;                   // transpose of P
    std::vector<double> cinv;    // dense inverse of L (coarsest level only), row-major
    HostCSR Dn;                  // (n_coarse x 2n) [R | -R L]: restricted residual from [b; x2]
    HostCSR Up;                  // (n x (2n + n_coarse)) [E | E P | w D^-1] on [x2; xc; b]: prolongation
                                 // and one smoothing sweep
};

// Structured triangulation of a union of square cells, Taylor-Hood P2/P1 numbering.
struct HostMesh {
    mhd_mesh_desc desc{};
    int nx = 0, ny = 0;          // cell grid
    double h = 0, x0 = 0, y0 = 0, xmax = 0;
    int nP2 = 0, nP1 = 0, n_el = 0;
    std::vector<double> xy;      // nP2 x 2
    std::vector<int32_t> tri;    // n_el x 6 P2 ids (v0,v1,v2,m01,m12,m20)
    std::vector<int32_t> tri1;   // n_el x 3 P1 ids
    std::vector<int32_t> p1_of_p2;  // P2 node -> P1 id (vertices) or -1
    std::vector<int32_t> hs_p2;  // half-step grid point (I, K) -> P2 id or -1, (2 ny + 1) x (2 nx + 1)
    std::vector<int32_t> cell_el;   // cell (i, k) -> its lower element (upper = +1) or -1, ny x nx
    std::vector<uint8_t> bnd;    // per P2 node: on the boundary
    std::vector<uint8_t> dir;    // per P2 node: Dirichlet
    std::vector<int32_t> dir_nodes;
    std::vector<uint8_t> pfix;   // per P1 node: fixed row of the pressure Laplacian (pin / outflow)
    int32_t pin = -1;
    // patterns of the saddle-point operator
    HostCSR A;                   // scalar P2 x P2 (pattern only)
    HostCSR Bt;                  // P2 x P1
    HostCSR B;                   // P1 x P2
    // element -> CSR slot maps and slot -> element contributions (deterministic gathers)
    std::vector<int32_t> slotA;  // n_el x 36
    std::vector<int32_t> permA, permBtB;     // transposition maps of the operator slots
    std::vector<int32_t> gA_ptr, gA_idx;     // nnz_A + 1, contributions e*36 + a*6 + b
    std::vector<int32_t> gB_ptr, gB_idx;     // nnz_B + 1, contributions e*18 + k*6 + a
    std::vector<int32_t> gBt_ptr, gBt_idx;   // nnz_Bt + 1, contributions e*18 + k*6 + a
    // P2 node -> (element, local index) incidence, sorted by element
    std::vector<int32_t> inc_ptr, inc;       // inc entry = e*8 + a
    std::vector<double> mp;      // lumped P1 mass (integral of each P1 basis function)
    std::vector<double> diagM, diagK;        // per P2 node
    HostCSR Bs, Bts;                         // divergence over velocity unknowns (BC rows applied)
    double schur_dt = -1.0, schur_nuc = -1.0;
    std::vector<HostLevel> levels;           // pressure Schur-approximation hierarchy
};

// Row tiles of the saddle-point operator for the LDS-staged kernels.  The
// mesh is cut into rectangles of tx x ty half-steps (the P2 node spacing); a
// tile owns the P2 rows and P1 rows whose nodes lie in its rectangle and
// stages every node value those rows read.  Empty rectangles are dropped.
struct HostTiling {
    int tx = 0, ty = 0;
    int ntiles = 0;
    int max_s2 = 0, max_s1 = 0;             // largest staged P2 / P1 node counts
    int max_r2 = 0, max_r1 = 0;             // largest owned P2 / P1 row counts
    std::vector<int32_t> r2_ptr, r2;        // tile -> owned P2 rows
    std::vector<int32_t> r2_self;           // per owned P2 row: local index of its own node
    std::vector<int32_t> r1_ptr, r1;        // tile -> owned P1 rows
    std::vector<int32_t> r1_self;           // per owned P1 row: local index of its own node
    std::vector<int32_t> s2_ptr, s2;        // tile -> staged P2 nodes (ascending)
    std::vector<int32_t> s1_ptr, s1;        // tile -> staged P1 nodes (ascending)
    std::vector<int32_t> a_loc, bt_loc, b_loc;   // per CSR entry of A, B^T, B: local column index
    // the entries again in tile order (rows as listed in r2 / r1): per entry the
    // local column index and the position of the entry in the global CSR arrays;
    // each row is padded to a multiple of 4 entries with (0, -1)
    std::vector<int32_t> ta_rp, ta_loc, ta_gp;   // over r2 (size |r2| + 1)
    std::vector<int32_t> tbt_rp, tbt_loc, tbt_gp;
    std::vector<int32_t> tb_rp, tb_loc, tb_gp;   // over r1
    int max_ea = 0, max_ebt = 0, max_eb = 0;     // largest per-tile entry counts
};
void build_tiling(const HostMesh& m, int tx, int ty, HostTiling& t);

// Row-per-lane tiles of the saddle-point operator (sliced ELL over LDS-staged
// node values).  Rectangles of tx x ty half-steps as above; a workgroup stages
// the values of M members of every node its rows read, then each lane
// computes one row.  A tile's P2 rows (sorted by entry counts, longest first)
// and its P1 rows are cut into blocks of 64, one wavefront each; a block's
// entries are stored column-major (entry k of all 64 lanes together), padded
// to the longest row of the block with (the first slot of the kind the entries
// read, CSR position -1).
constexpr int ell_p2_bytes(int M) { return 8 * M + 16; }   // LDS bytes per staged P2 node: 2 x M floats + 16 padding
constexpr int ell_p1_bytes(int M) { return 4 * M + 16; }   // LDS bytes per staged P1 node: M floats + 16 padding
struct HostEll {
    int tx = 0, ty = 0, m = 0, ntiles = 0;
    int max_lds = 0;                 // largest staged bytes of a tile
    int max_lds1 = 0;                // largest staged bytes of a tile's P1 nodes alone
    int max_lds2 = 0;                // largest staged bytes of a tile's P2 nodes alone
    int max_blocks = 0;              // largest number of row blocks of a tile
    int max_blocks2 = 0;             // largest number of P2 row blocks of a tile (they come first)
    int max_k = 0;                   // longest row
    std::vector<int32_t> tile;       // 8 per tile: s2 offset, s2 count, s1 offset, s1 count, first block, blocks
    std::vector<int32_t> s2, s1;     // staged P2 / P1 nodes of every tile (ascending within a tile)
    std::vector<int32_t> blk;        // 8 per block: kind (0 P2, 1 P1), rows, K1, K2, entries 1, entries 2, row offset
    std::vector<int32_t> rows;       // 64 per block: row (P2 node or P1 node) or -1
    std::vector<int32_t> self;       // 64 per block: LDS offset of the row's own node
    std::vector<int32_t> loc;        // per entry: LDS byte offset of the staged node it reads
    std::vector<int32_t> gp;         // per entry: position in the CSR value arrays, -1 for padding
};
// P2 blocks: entries 1 are A (K1 per lane), entries 2 are B^T (K2); P1 blocks: entries 1 are B.
void build_ell(const HostMesh& m, int tx, int ty, int M, HostEll& t);

mhd_status build_mesh(const mhd_mesh_desc* d, HostMesh& m, bool full);
mhd_status schur_values(HostMesh& m, double dt, double nu_c);
void mesh_counts(const HostMesh& m, mhd_mesh_info* info);

// reference-element tables (uploaded to constant memory; also compile-time constants below)
struct RefTables {
    double w[7];            // quadrature weights summing to 1
    double phi[7][6];       // P2 values at the points
    double dphi[7][6][2];   // reference gradients
    double psi[7][3];       // P1 values
    double Mhat[6][6];      // int_ref phi_a phi_b (area 1/2)
    double Khat[6][6][2][2];// int_ref d_e phi_a d_f phi_b
    double That[6][6][6][2];// int_ref phi_a phi_b d_e phi_c
    double Shat[6][6][6][2];// (That[a][b][c] - That[c][b][a]) / 2
    double Bhat[3][6][2];   // -int_ref psi_k d_e phi_a
    double Kc[6][6][3];     // Khat[a][b] combined for a symmetric G: [0][0], [0][1] + [1][0], [1][1]
};
void make_ref_tables(RefTables& t);

// square root by Newton's iteration, usable in constant expressions
constexpr double ce_sqrt(double x) {
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 100; ++i) r = 0.5 * (r + x / r);
    return r;
}

// The reference-element tables of the P2-P1 pair (Section 2), evaluated with
// Radon's 7-point rule, exact for the polynomial degrees involved (mass: 4,
// stiffness: 2, trilinear: 5).  constexpr, so that kernels can take the
// entries as immediate constants.
constexpr RefTables build_ref_tables() {
    RefTables t{};
    const double s15 = ce_sqrt(15.0);
    double lam[7][3] = {};
    lam[0][0] = lam[0][1] = lam[0][2] = 1.0 / 3.0;
    t.w[0] = 9.0 / 40.0;
    const double aa[2] = {(6.0 - s15) / 21.0, (6.0 + s15) / 21.0};
    const double ww[2] = {(155.0 - s15) / 1200.0, (155.0 + s15) / 1200.0};
    int q = 1;
    for (int o = 0; o < 2; ++o) {
        const double a = aa[o], b = 1.0 - 2.0 * a;
        const double pts[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
        for (int k = 0; k < 3; ++k) {
            for (int i = 0; i < 3; ++i) lam[q][i] = pts[k][i];
            t.w[q] = ww[o];
            ++q;
        }
    }
    // barycentric gradients on the reference triangle (0,0),(1,0),(0,1); local
    // nodes: the three vertices, then the midpoints of edges 01, 12, 20
    const double dl[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    const int ed[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (q = 0; q < 7; ++q) {
        for (int i = 0; i < 3; ++i) {
            const double li = lam[q][i];
            t.phi[q][i] = li * (2.0 * li - 1.0);
            for (int d = 0; d < 2; ++d) t.dphi[q][i][d] = (4.0 * li - 1.0) * dl[i][d];
            t.psi[q][i] = li;
        }
        for (int e = 0; e < 3; ++e) {
            const int a = ed[e][0], b = ed[e][1];
            t.phi[q][3 + e] = 4.0 * lam[q][a] * lam[q][b];
            for (int d = 0; d < 2; ++d) t.dphi[q][3 + e][d] = 4.0 * (lam[q][b] * dl[a][d] + lam[q][a] * dl[b][d]);
        }
    }
    for (q = 0; q < 7; ++q) {
        const double wq = 0.5 * t.w[q];
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                t.Mhat[a][b] += wq * t.phi[q][a] * t.phi[q][b];
                for (int e = 0; e < 2; ++e)
                    for (int f = 0; f < 2; ++f) t.Khat[a][b][e][f] += wq * t.dphi[q][a][e] * t.dphi[q][b][f];
                for (int c = 0; c < 6; ++c)
                    for (int e = 0; e < 2; ++e) t.That[a][b][c][e] += wq * t.phi[q][a] * t.phi[q][b] * t.dphi[q][c][e];
            }
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 6; ++a)
                for (int e = 0; e < 2; ++e) t.Bhat[k][a][e] -= wq * t.psi[q][k] * t.dphi[q][a][e];
    }
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b)
            for (int c = 0; c < 6; ++c)
                for (int e = 0; e < 2; ++e) t.Shat[a][b][c][e] = 0.5 * (t.That[a][b][c][e] - t.That[c][b][a][e]);
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            t.Kc[a][b][0] = t.Khat[a][b][0][0];
            t.Kc[a][b][1] = t.Khat[a][b][0][1] + t.Khat[a][b][1][0];
            t.Kc[a][b][2] = t.Khat[a][b][1][1];
        }
    return t;
}

}  // namespace mhd
