// Host-side invariants of the row-per-lane (sliced ELL) tilings of the
// saddle-point operator, checked against the CSR patterns they are built from:
// every row is owned by exactly one tile and lane; every entry of a row appears
// at its CSR position in its block's column-major entry list and points at the
// LDS slot that holds its column's node; padding entries point at the first
// slot of the kind they read and carry no CSR position; every LDS access stays
// inside the tile's staged bytes; P2 blocks precede the P1 blocks of a tile.
// Built and run by tests/test_tiling_host.py.
#include <algorithm>
#include <vector>
#include <cstdio>
#include <cassert>
#include <cstdlib>
#include "common.h"
namespace mhd { void set_error(const std::string&) {} std::string hip_error_string(int){return "";} }
using namespace mhd;
#define REQ(c) do { if (!(c)) { printf("FAIL %s line %d\n", #c, __LINE__); exit(1); } } while (0)
int main() {
    int sizes[][3] = {{0, 128, 0}, {0, 12, 0}, {0, 3, 0}, {1, 4, 1}};   // unit square N, step channel m
    for (auto& sz : sizes) {
        mhd_mesh_desc d{sz[0], sz[1], sz[2]};
        HostMesh m;
        if (build_mesh(&d, m, true) != MHD_OK) { printf("mesh fail\n"); return 1; }
        int shapes[][3] = {{16,8,16},{16,16,16},{32,8,16},{16,8,8},{16,16,8},{32,8,8}};
        for (auto& sh : shapes) {
            HostEll t;
            build_ell(m, sh[0], sh[1], sh[2], t);
            const int kEllP2Bytes = ell_p2_bytes(sh[2]), kEllP1Bytes = ell_p1_bytes(sh[2]), kEllM = sh[2];
            std::vector<int> seen2(m.nP2, 0), seen1(m.nP1, 0);
            long useful = 0, padded = 0;
            REQ((int)t.tile.size() == 8 * t.ntiles);
            for (int T = 0; T < t.ntiles; ++T) {
                const int* td = &t.tile[8 * T];
                const int s2o = td[0], n2 = td[1], s1o = td[2], n1 = td[3], b0 = td[4], nb = td[5];
                const int lds = n2 * kEllP2Bytes + n1 * kEllP1Bytes;
                REQ(lds <= t.max_lds && nb <= t.max_blocks && nb >= 1);
                REQ(n2 * kEllP2Bytes <= t.max_lds2 && n1 * kEllP1Bytes <= t.max_lds1);
                { int nb2 = 0; for (int b = b0; b < b0 + nb; ++b) { if (t.blk[8*b] == 0) { REQ(b - b0 == nb2); nb2++; } } REQ(nb2 <= t.max_blocks2); }
                REQ(s2o + n2 <= (int)t.s2.size() && s1o + n1 <= (int)t.s1.size());
                auto node_at = [&](int off, int& kind) -> int {
                    if (off < n2 * kEllP2Bytes) { REQ(off % kEllP2Bytes == 0); kind = 2; return t.s2[s2o + off / kEllP2Bytes]; }
                    int o = off - n2 * kEllP2Bytes; REQ(o % kEllP1Bytes == 0 && o / kEllP1Bytes < n1); kind = 1; return t.s1[s1o + o / kEllP1Bytes];
                };
                for (int b = b0; b < b0 + nb; ++b) {
                    REQ(b * 8 + 8 <= (int)t.blk.size());
                    const int* bd = &t.blk[8 * b];
                    const int kind = bd[0], nr = bd[1], K1 = bd[2], K2 = bd[3], e1 = bd[4], e2 = bd[5], ro = bd[6];
                    REQ(nr >= 1 && nr <= 64 && K1 <= t.max_k && K2 <= t.max_k);
                    REQ(e2 == e1 + 64 * K1 && e2 + 64 * K2 <= (int)t.loc.size() && ro + 64 <= (int)t.rows.size());
                    for (int l = 0; l < 64; ++l) {
                        const int row = t.rows[ro + l];
                        REQ((l < nr) == (row >= 0));
                        for (int k = 0; k < K1 + K2; ++k) {
                            const int e = (k < K1 ? e1 + 64 * k : e2 + 64 * (k - K1)) + l;
                            REQ(t.loc[e] >= 0 && t.loc[e] + (k < K1 || kind == 1 ? 2 * kEllM * 4 : kEllM * 4) <= lds);
                            padded++;
                        }
                        if (row < 0) continue;
                        const HostCSR& c1 = kind == 0 ? m.A : m.B;
                        const int n1r = c1.rowptr[row + 1] - c1.rowptr[row];
                        REQ(n1r <= K1);
                        for (int k = 0; k < K1; ++k) {
                            const int e = e1 + 64 * k + l;
                            if (k < n1r) {
                                REQ(t.gp[e] == c1.rowptr[row] + k);
                                int nk; REQ(node_at(t.loc[e], nk) == c1.col[t.gp[e]] && nk == 2);
                                useful++;
                            } else REQ(t.gp[e] == -1 && t.loc[e] == 0);
                        }
                        if (kind == 0) {
                            seen2[row]++;
                            { int nk; REQ(node_at(t.self[ro + l], nk) == row && nk == 2); }
                            const int n2r = m.Bt.rowptr[row + 1] - m.Bt.rowptr[row];
                            REQ(n2r <= K2);
                            for (int k = 0; k < K2; ++k) {
                                const int e = e2 + 64 * k + l;
                                if (k < n2r) {
                                    REQ(t.gp[e] == m.Bt.rowptr[row] + k);
                                    int nk; REQ(node_at(t.loc[e], nk) == m.Bt.col[t.gp[e]] && nk == 1);
                                    useful++;
                                } else REQ(t.gp[e] == -1 && t.loc[e] == n2 * kEllP2Bytes);
                            }
                        } else {
                            seen1[row]++;
                            REQ(K2 == 0);
                            int nk; REQ(node_at(t.self[ro + l], nk) == row && nk == 1);
                        }
                    }
                }
            }
            for (int i = 0; i < m.nP2; ++i) REQ(seen2[i] == 1);
            for (int i = 0; i < m.nP1; ++i) REQ(seen1[i] == 1);
            printf("M %d kind %d N %3d %2dx%2d tiles %6d lds %6d B blocks %d max_k %d  entries useful %ld padded %ld (%.2f)\n",
                   sh[2], sz[0], sz[1], sh[0], sh[1], t.ntiles, t.max_lds, t.max_blocks, t.max_k, useful, padded, (double)padded / useful);
        }
    }
    return 0;
}
