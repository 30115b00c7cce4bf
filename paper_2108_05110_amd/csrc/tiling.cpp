// Row tiles of the saddle-point operator for the LDS-staged SpMM and Jacobi
// kernels (host side): CSR-order tiles and row-per-lane (sliced ELL) tiles.  Rows are grouped by the rectangle of tx x ty
// half-steps their node lies in; each tile lists the node values its rows read
// (the union of their column indices), and every CSR entry gets the position
// of its column in its row's tile list.
#include <algorithm>
#include <cmath>
#include <tuple>

#include "common.h"

namespace mhd {

namespace {
// pads a row of tile-ordered entries to a multiple of 4 with (local column 0,
// no global entry): the LDS-staged kernels read a row 4 entries at a time
void pad4(std::vector<int32_t>& loc, std::vector<int32_t>& gp) {
    while (loc.size() % 4) {
        loc.push_back(0);
        gp.push_back(-1);
    }
}
}  // namespace

void build_tiling(const HostMesh& m, int tx, int ty, HostTiling& t) {
    t = HostTiling{};
    t.tx = tx;
    t.ty = ty;
    const int nP2 = m.nP2, nP1 = m.nP1;
    // half-step coordinates and rectangle of every P2 node
    int hxmax = 0, hymax = 0;
    std::vector<int> hx(nP2), hy(nP2);
    for (int i = 0; i < nP2; ++i) {
        hx[i] = (int)std::lround(2.0 * (m.xy[2 * (size_t)i] - m.x0) / m.h);
        hy[i] = (int)std::lround(2.0 * (m.xy[2 * (size_t)i + 1] - m.y0) / m.h);
        hxmax = std::max(hxmax, hx[i]);
        hymax = std::max(hymax, hy[i]);
    }
    const int gx = hxmax / tx + 1, gy = hymax / ty + 1;
    std::vector<int> rect(nP2);
    for (int i = 0; i < nP2; ++i) rect[i] = (hy[i] / ty) * gx + hx[i] / tx;
    std::vector<int32_t> p2_of_p1(nP1, -1);
    for (int i = 0; i < nP2; ++i)
        if (m.p1_of_p2[i] >= 0) p2_of_p1[m.p1_of_p2[i]] = i;
    // rows of every rectangle, ascending
    std::vector<std::vector<int32_t>> rows2((size_t)gx * gy), rows1((size_t)gx * gy);
    for (int i = 0; i < nP2; ++i) rows2[rect[i]].push_back(i);
    for (int k = 0; k < nP1; ++k) rows1[rect[p2_of_p1[k]]].push_back(k);

    t.a_loc.assign(m.A.col.size(), 0);
    t.bt_loc.assign(m.Bt.col.size(), 0);
    t.b_loc.assign(m.B.col.size(), 0);
    t.r2_ptr.push_back(0);
    t.r1_ptr.push_back(0);
    t.ta_rp.push_back(0);
    t.tbt_rp.push_back(0);
    t.tb_rp.push_back(0);
    t.s2_ptr.push_back(0);
    t.s1_ptr.push_back(0);
    std::vector<int32_t> loc2(nP2, -1), loc1(nP1, -1);
    std::vector<int32_t> st2, st1;
    for (size_t r = 0; r < rows2.size(); ++r) {
        const auto& R2 = rows2[r];
        const auto& R1 = rows1[r];
        if (R2.empty() && R1.empty()) continue;
        st2.clear();
        st1.clear();
        for (int32_t u : R2) {
            for (int32_t p = m.A.rowptr[u]; p < m.A.rowptr[u + 1]; ++p) st2.push_back(m.A.col[p]);
            for (int32_t p = m.Bt.rowptr[u]; p < m.Bt.rowptr[u + 1]; ++p) st1.push_back(m.Bt.col[p]);
            st2.push_back(u);
        }
        for (int32_t k : R1) {
            for (int32_t q = m.B.rowptr[k]; q < m.B.rowptr[k + 1]; ++q) st2.push_back(m.B.col[q]);
            st1.push_back(k);
        }
        std::sort(st2.begin(), st2.end());
        st2.erase(std::unique(st2.begin(), st2.end()), st2.end());
        std::sort(st1.begin(), st1.end());
        st1.erase(std::unique(st1.begin(), st1.end()), st1.end());
        for (size_t s = 0; s < st2.size(); ++s) loc2[st2[s]] = (int32_t)s;
        for (size_t s = 0; s < st1.size(); ++s) loc1[st1[s]] = (int32_t)s;
        const size_t ea0 = t.ta_loc.size(), ebt0 = t.tbt_loc.size(), eb0 = t.tb_loc.size();
        for (int32_t u : R2) {
            for (int32_t p = m.A.rowptr[u]; p < m.A.rowptr[u + 1]; ++p) {
                t.a_loc[p] = loc2[m.A.col[p]];
                t.ta_loc.push_back(t.a_loc[p]);
                t.ta_gp.push_back(p);
            }
            pad4(t.ta_loc, t.ta_gp);
            for (int32_t p = m.Bt.rowptr[u]; p < m.Bt.rowptr[u + 1]; ++p) {
                t.bt_loc[p] = loc1[m.Bt.col[p]];
                t.tbt_loc.push_back(t.bt_loc[p]);
                t.tbt_gp.push_back(p);
            }
            pad4(t.tbt_loc, t.tbt_gp);
            t.ta_rp.push_back((int32_t)t.ta_loc.size());
            t.tbt_rp.push_back((int32_t)t.tbt_loc.size());
            t.r2.push_back(u);
            t.r2_self.push_back(loc2[u]);
        }
        for (int32_t k : R1) {
            for (int32_t q = m.B.rowptr[k]; q < m.B.rowptr[k + 1]; ++q) {
                t.b_loc[q] = loc2[m.B.col[q]];
                t.tb_loc.push_back(t.b_loc[q]);
                t.tb_gp.push_back(q);
            }
            pad4(t.tb_loc, t.tb_gp);
            t.tb_rp.push_back((int32_t)t.tb_loc.size());
            t.r1.push_back(k);
            t.r1_self.push_back(loc1[k]);
        }
        t.max_ea = std::max(t.max_ea, (int)(t.ta_loc.size() - ea0));
        t.max_ebt = std::max(t.max_ebt, (int)(t.tbt_loc.size() - ebt0));
        t.max_eb = std::max(t.max_eb, (int)(t.tb_loc.size() - eb0));
        t.s2.insert(t.s2.end(), st2.begin(), st2.end());
        t.s1.insert(t.s1.end(), st1.begin(), st1.end());
        t.r2_ptr.push_back((int32_t)t.r2.size());
        t.r1_ptr.push_back((int32_t)t.r1.size());
        t.s2_ptr.push_back((int32_t)t.s2.size());
        t.s1_ptr.push_back((int32_t)t.s1.size());
        t.max_s2 = std::max(t.max_s2, (int)st2.size());
        t.max_s1 = std::max(t.max_s1, (int)st1.size());
        t.max_r2 = std::max(t.max_r2, (int)R2.size());
        t.max_r1 = std::max(t.max_r1, (int)R1.size());
        ++t.ntiles;
    }
}

void build_ell(const HostMesh& m, int tx, int ty, int M, HostEll& t) {
    t = HostEll{};
    t.tx = tx;
    t.ty = ty;
    t.m = M;
    const int P2B = ell_p2_bytes(M), P1B = ell_p1_bytes(M);
    const int nP2 = m.nP2, nP1 = m.nP1;
    int hxmax = 0;
    std::vector<int> hx(nP2), hy(nP2);
    for (int i = 0; i < nP2; ++i) {
        hx[i] = (int)std::lround(2.0 * (m.xy[2 * (size_t)i] - m.x0) / m.h);
        hy[i] = (int)std::lround(2.0 * (m.xy[2 * (size_t)i + 1] - m.y0) / m.h);
        hxmax = std::max(hxmax, hx[i]);
    }
    const int gx = hxmax / tx + 1;
    int nrect = 0;
    std::vector<int> rect(nP2);
    for (int i = 0; i < nP2; ++i) {
        rect[i] = (hy[i] / ty) * gx + hx[i] / tx;
        nrect = std::max(nrect, rect[i] + 1);
    }
    std::vector<int32_t> p2_of_p1(nP1, -1);
    for (int i = 0; i < nP2; ++i)
        if (m.p1_of_p2[i] >= 0) p2_of_p1[m.p1_of_p2[i]] = i;
    std::vector<std::vector<int32_t>> rows2(nrect), rows1(nrect);
    for (int i = 0; i < nP2; ++i) rows2[rect[i]].push_back(i);
    for (int k = 0; k < nP1; ++k) rows1[rect[p2_of_p1[k]]].push_back(k);
    auto len = [](const HostCSR& c, int r) { return c.rowptr[r + 1] - c.rowptr[r]; };
    std::vector<int32_t> off2(nP2, -1), off1(nP1, -1);
    std::vector<int32_t> st2, st1;
    for (int r = 0; r < nrect; ++r) {
        std::vector<int32_t> R2 = rows2[r], R1 = rows1[r];
        if (R2.empty() && R1.empty()) continue;
        st2.clear();
        st1.clear();
        for (int32_t u : R2) {
            for (int32_t p = m.A.rowptr[u]; p < m.A.rowptr[u + 1]; ++p) st2.push_back(m.A.col[p]);
            for (int32_t p = m.Bt.rowptr[u]; p < m.Bt.rowptr[u + 1]; ++p) st1.push_back(m.Bt.col[p]);
        }
        for (int32_t k : R1) {
            for (int32_t q = m.B.rowptr[k]; q < m.B.rowptr[k + 1]; ++q) st2.push_back(m.B.col[q]);
            st1.push_back(k);
        }
        // staged P2 nodes by (line, parity of the position along the line, position): the
        // same-kind nodes a lane's neighbours read lie 2 half-steps apart and so get
        // consecutive slots, whose padded LDS rows start in different banks
        auto key = [&](int32_t u) { return std::make_tuple(hy[u], hx[u] & 1, hx[u]); };
        std::sort(st2.begin(), st2.end());
        st2.erase(std::unique(st2.begin(), st2.end()), st2.end());
        std::sort(st2.begin(), st2.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        std::sort(st1.begin(), st1.end());
        st1.erase(std::unique(st1.begin(), st1.end()), st1.end());
        const int p1base = (int)st2.size() * P2B;
        for (size_t s = 0; s < st2.size(); ++s) off2[st2[s]] = (int32_t)s * P2B;
        for (size_t s = 0; s < st1.size(); ++s) off1[st1[s]] = p1base + (int32_t)s * P1B;
        t.max_lds = std::max(t.max_lds, p1base + (int)st1.size() * P1B);
        t.max_lds1 = std::max(t.max_lds1, (int)st1.size() * P1B);
        t.max_lds2 = std::max(t.max_lds2, p1base);
        t.max_blocks2 = std::max(t.max_blocks2, (int)((R2.size() + 63) / 64));
        // longest rows first, so that the rows of a block have similar lengths
        std::stable_sort(R2.begin(), R2.end(), [&](int32_t a, int32_t b) {
            const int la = len(m.A, a), lb = len(m.A, b);
            if (la != lb) return la > lb;
            const int ba = len(m.Bt, a), bb = len(m.Bt, b);
            return ba != bb ? ba > bb : key(a) < key(b);
        });
        std::stable_sort(R1.begin(), R1.end(), [&](int32_t a, int32_t b) { return len(m.B, a) > len(m.B, b); });
        const int first = (int)(t.blk.size() / 8);
        auto add_blocks = [&](const std::vector<int32_t>& R, int kind) {
            for (size_t b0 = 0; b0 < R.size(); b0 += 64) {
                const int nr = (int)std::min<size_t>(64, R.size() - b0);
                const HostCSR& c1 = kind == 0 ? m.A : m.B;
                int K1 = 0, K2 = 0;
                for (int l = 0; l < nr; ++l) {
                    K1 = std::max(K1, len(c1, R[b0 + l]));
                    if (kind == 0) K2 = std::max(K2, len(m.Bt, R[b0 + l]));
                }
                t.max_k = std::max(t.max_k, std::max(K1, K2));
                const int e1 = (int)t.loc.size(), e2 = e1 + 64 * K1, ro = (int)t.rows.size();
                t.blk.insert(t.blk.end(), {kind, nr, K1, K2, e1, e2, ro, 0});
                t.loc.resize((size_t)e2, 0);                      // padding reads the first P2 slot
                t.loc.resize((size_t)e2 + 64 * K2, p1base);       // ... or the first P1 slot
                t.gp.resize((size_t)e2 + 64 * K2, -1);
                for (int l = 0; l < 64; ++l) {
                    const int32_t row = l < nr ? R[b0 + l] : -1;
                    t.rows.push_back(row);
                    t.self.push_back(row < 0 ? 0 : kind == 1 ? off1[row] : off2[row]);
                    if (row < 0) continue;
                    for (int32_t p = c1.rowptr[row], k = 0; p < c1.rowptr[row + 1]; ++p, ++k) {
                        t.loc[(size_t)e1 + 64 * k + l] = off2[c1.col[p]];
                        t.gp[(size_t)e1 + 64 * k + l] = p;
                    }
                    if (kind == 0)
                        for (int32_t p = m.Bt.rowptr[row], k = 0; p < m.Bt.rowptr[row + 1]; ++p, ++k) {
                            t.loc[(size_t)e2 + 64 * k + l] = off1[m.Bt.col[p]];
                            t.gp[(size_t)e2 + 64 * k + l] = p;
                        }
                }
            }
        };
        add_blocks(R2, 0);
        add_blocks(R1, 1);
        const int nblk = (int)(t.blk.size() / 8) - first;
        t.max_blocks = std::max(t.max_blocks, nblk);
        t.tile.insert(t.tile.end(), {(int32_t)t.s2.size(), (int32_t)st2.size(), (int32_t)t.s1.size(),
                                     (int32_t)st1.size(), first, nblk, 0, 0});
        t.s2.insert(t.s2.end(), st2.begin(), st2.end());
        t.s1.insert(t.s1.end(), st1.begin(), st1.end());
        ++t.ntiles;
    }
}

}  // namespace mhd
