// Assembly kernels of libmhd_ens (gfx950):
//   ensemble statistics (mean over members, eddy-viscosity length l^2 at the
//   quadrature points), shared saddle-point matrix of one subproblem, constant
//   mass/stiffness/divergence matrices, and the batched per-member right-hand
//   sides of Algorithm 1 (paper, Section 3, (weaknew1)/(weaknew2)).
//
// Layouts: member blocks are row-major with the member index fastest, so the
// J values of one node component are contiguous and a group of JP lanes
// (JP = power of two >= min(J, 64)) reads them coalesced.  All reductions are
// fixed-order (lane butterflies, per-slot gather lists): results are
// bitwise reproducible run to run; there are no floating-point atomics.
#include <hip/hip_runtime.h>

#include "device.h"

namespace mhd {

__constant__ RefTables c_ref;

void upload_ref_tables(const RefTables& t) { (void)hipMemcpyToSymbol(HIP_SYMBOL(c_ref), &t, sizeof(RefTables)); }

namespace {

constexpr int kBlock = 256;

// Hardware dispatches workgroup b to XCD b % 8.  Give XCD x a contiguous range
// of logical blocks so neighbouring rows (which share gathered operands) are
// served from the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    int64_t q = G >> 3, r = G & 7, x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

struct Lanes {
    int JP, sub, j0;
    int64_t unit;
};

__device__ __forceinline__ Lanes lanes(int JP) {
    Lanes L;
    int lane = threadIdx.x & 63;
    int wave = threadIdx.x >> 6;
    int rpw = 64 / JP;
    L.JP = JP;
    L.sub = lane / JP;
    L.j0 = lane % JP;
    int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    L.unit = (blk * (kBlock / 64) + wave) * rpw + L.sub;
    return L;
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int JP) {
    for (int off = JP >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double group_max(double v, int JP) {
    for (int off = JP >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// lanes per unit (row or element): the power of two >= J, at most cap (16: a
// wavefront takes four or more units and a lane several members)
inline int pick_jp(int J, int cap = 16) {
    int p = 1;
    while (p < J && p < cap) p <<= 1;
    return p;
}

inline unsigned grid_for(int64_t units, int JP) {
    int64_t per_block = (kBlock / 64) * (64 / JP);
    return (unsigned)((units + per_block - 1) / per_block);
}

// -------------------------------------------------------------- (a1) ensemble mean
__global__ void __launch_bounds__(kBlock) k_mean(const double* __restrict__ z, double* __restrict__ zbar,
                                                 int64_t rows, int J, int JP) {
    Lanes L = lanes(JP);
    double acc = 0.0;
    if (L.unit < rows)
        for (int j = L.j0; j < J; j += JP) acc += z[L.unit * J + j];
    acc = group_sum(acc, JP);
    if (L.unit < rows && L.j0 == 0) zbar[L.unit] = acc / (double)J;
}

// -------------------------------------------------------------- (a1) l^2 = max_j |z_j'(x_q)|^2
__global__ void __launch_bounds__(kBlock) k_eddy_l2(const int32_t* __restrict__ tri, const double* __restrict__ z,
                                                    const double* __restrict__ zbar, double* __restrict__ l2,
                                                    int n_el, int J, int JP) {
    Lanes L = lanes(JP);
    double mx[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) mx[q] = 0.0;
    if (L.unit < n_el) {
        int t[6];
        double zb[6][2];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            t[a] = tri[L.unit * 6 + a];
            zb[a][0] = zbar[2 * t[a]];
            zb[a][1] = zbar[2 * t[a] + 1];
        }
        for (int j = L.j0; j < J; j += JP) {
            double zv[6][2];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                zv[a][0] = z[(int64_t)(2 * t[a]) * J + j] - zb[a][0];
                zv[a][1] = z[(int64_t)(2 * t[a] + 1) * J + j] - zb[a][1];
            }
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                double ux = 0.0, uy = 0.0;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    ux += c_ref.phi[q][a] * zv[a][0];
                    uy += c_ref.phi[q][a] * zv[a][1];
                }
                mx[q] = fmax(mx[q], ux * ux + uy * uy);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) mx[q] = group_max(mx[q], JP);
    if (L.unit < n_el && L.j0 == 0)
        for (int q = 0; q < 7; ++q) l2[L.unit * 7 + q] = mx[q];
}

// -------------------------------------------------------------- element geometry helpers
struct Geo {
    double det, Ji[2][2], G[2][2];
};

__device__ __forceinline__ Geo load_geo(const double* geo, int64_t e) {
    Geo g;
    g.det = geo[e * 6];
    g.Ji[0][0] = geo[e * 6 + 1];
    g.Ji[0][1] = geo[e * 6 + 2];
    g.Ji[1][0] = geo[e * 6 + 3];
    g.Ji[1][1] = geo[e * 6 + 4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) g.G[a][b] = g.Ji[a][0] * g.Ji[b][0] + g.Ji[a][1] * g.Ji[b][1];
    return g;
}

// -------------------------------------------------------------- (a2) element matrices of A
// A_e = M_e/dt + nu_c K_e + N_e(<z>) + K_e[2 mu dt l^2]   (6 x 6 scalar, per element)
__global__ void __launch_bounds__(kBlock) k_elem_A(const int32_t* __restrict__ tri, const double* __restrict__ geo,
                                                   const double* __restrict__ zbar, const double* __restrict__ l2,
                                                   double* __restrict__ elem, int n_el, double inv_dt, double nu_c,
                                                   double eddy_c, int convective) {
    int64_t e = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (e >= n_el) return;
    Geo g = load_geo(geo, e);
    double zh[6][2];
    for (int b = 0; b < 6; ++b) {
        int t = tri[e * 6 + b];
        double z0 = zbar[2 * t], z1 = zbar[2 * t + 1];
        zh[b][0] = g.det * (g.Ji[0][0] * z0 + g.Ji[0][1] * z1);
        zh[b][1] = g.det * (g.Ji[1][0] * z0 + g.Ji[1][1] * z1);
    }
    double kap[7];
    for (int q = 0; q < 7; ++q) kap[q] = 0.5 * g.det * c_ref.w[q] * eddy_c * l2[e * 7 + q];
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 6; ++c) {
            double v = g.det * c_ref.Mhat[a][c] * inv_dt;
            double k = 0.0;
            for (int p = 0; p < 2; ++p)
                for (int r = 0; r < 2; ++r) k += c_ref.Khat[a][c][p][r] * g.G[p][r];
            v += nu_c * g.det * k;
            double cv = 0.0;
            for (int b = 0; b < 6; ++b)
                for (int p = 0; p < 2; ++p)
                    cv += (convective ? c_ref.That[a][b][c][p] : c_ref.Shat[a][b][c][p]) * zh[b][p];
            v += cv;
            double ed = 0.0;
            for (int q = 0; q < 7; ++q) {
                double s = 0.0;
                for (int p = 0; p < 2; ++p)
                    for (int r = 0; r < 2; ++r) s += c_ref.dphi[q][a][p] * c_ref.dphi[q][c][r] * g.G[p][r];
                ed += kap[q] * s;
            }
            elem[e * 36 + a * 6 + c] = v + ed;
        }
}

// Deterministic gather of element contributions into the CSR values of A;
// Dirichlet rows become identity rows.  Also records 1/diag(A).
__global__ void __launch_bounds__(kBlock) k_gather_A(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ gptr, const int32_t* __restrict__ gidx,
                                                     const uint8_t* __restrict__ dir, const double* __restrict__ elem,
                                                     double* __restrict__ val, float* __restrict__ val32,
                                                     double* __restrict__ dinv, float* __restrict__ dinv32, int nrows) {
    int64_t r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (r >= nrows) return;
    bool d = dir[r] != 0;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
        double v = 0.0;
        if (d) {
            v = (col[p] == r) ? 1.0 : 0.0;
        } else {
            for (int32_t q = gptr[p]; q < gptr[p + 1]; ++q) v += elem[gidx[q]];
        }
        val[p] = v;
        val32[p] = (float)v;
        if (col[p] == r) {
            dinv[r] = 1.0 / v;
            dinv32[r] = (float)(1.0 / v);
        }
    }
}

// -------------------------------------------------------------- constant matrices (once per mesh)
// elembuf per element: [0,36) mass, [36,72) stiffness, [72,108) divergence (k*12 + a*2 + d)
__global__ void __launch_bounds__(kBlock) k_elem_const(const double* __restrict__ geo, double* __restrict__ eb, int n_el) {
    int64_t e = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (e >= n_el) return;
    Geo g = load_geo(geo, e);
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 6; ++c) {
            eb[e * 108 + a * 6 + c] = g.det * c_ref.Mhat[a][c];
            double k = 0.0;
            for (int p = 0; p < 2; ++p)
                for (int r = 0; r < 2; ++r) k += c_ref.Khat[a][c][p][r] * g.G[p][r];
            eb[e * 108 + 36 + a * 6 + c] = g.det * k;
        }
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 6; ++a)
            for (int d = 0; d < 2; ++d) {
                double v = 0.0;
                for (int p = 0; p < 2; ++p) v += c_ref.Bhat[k][a][p] * g.Ji[p][d];
                eb[e * 108 + 72 + (k * 6 + a) * 2 + d] = g.det * v;
            }
}

__global__ void __launch_bounds__(kBlock) k_gather_MK(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ gptr,
                                                      const int32_t* __restrict__ gidx, const double* __restrict__ eb,
                                                      double* __restrict__ valM, double* __restrict__ valK, int nrows) {
    int64_t r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (r >= nrows) return;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
        double m = 0.0, k = 0.0;
        for (int32_t q = gptr[p]; q < gptr[p + 1]; ++q) {
            int32_t c = gidx[q];
            int64_t e = c / 36, ab = c % 36;
            m += eb[e * 108 + ab];
            k += eb[e * 108 + 36 + ab];
        }
        valM[p] = m;
        valK[p] = k;
    }
}

// gather of divergence contributions; rows flagged in `zero_row` are zeroed
__global__ void __launch_bounds__(kBlock) k_gather_B(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ gptr,
                                                     const int32_t* __restrict__ gidx, const double* __restrict__ eb,
                                                     const uint8_t* __restrict__ zero_row, int pin_row,
                                                     double* __restrict__ val, float* __restrict__ val32, int nrows) {
    int64_t r = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (r >= nrows) return;
    bool z = (zero_row && zero_row[r]) || (r == pin_row);
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
        double v0 = 0.0, v1 = 0.0;
        if (!z)
            for (int32_t q = gptr[p]; q < gptr[p + 1]; ++q) {
                int32_t c = gidx[q];
                int64_t e = c / 18, ka = c % 18;
                v0 += eb[e * 108 + 72 + ka * 2];
                v1 += eb[e * 108 + 72 + ka * 2 + 1];
            }
        val[2 * p] = v0;
        val[2 * p + 1] = v1;
        val32[2 * p] = (float)v0;
        val32[2 * p + 1] = (float)v1;
    }
}

// -------------------------------------------------------------- (a3) batched right-hand sides
// coef[j] = (nu_j - nu_m,j)/2, coef[J + j] = (nu_j' + nu_m,j')/2
__global__ void k_member_coefs(const double* __restrict__ nu, const double* __restrict__ nu_m, int J,
                               double* __restrict__ coef) {
    __shared__ double s_nu, s_nm;
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < J; ++j) {
            a += nu[j];
            b += nu_m[j];
        }
        s_nu = a / J;
        s_nm = b / J;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
        coef[j] = 0.5 * (nu[j] - nu_m[j]);
        coef[J + j] = 0.5 * ((nu[j] - s_nu) + (nu_m[j] - s_nm));
    }
}

// -------------------------------------------------------------- (a3) right-hand sides in one pass
// Every wavefront owns a strip of the structured cell grid and a slice of M
// members.  Its lanes are SLOTS = 64 / M element slots of M members each; a
// slot computes one element's 6 x 2 local rows for its members,
//   r = M_e (self/dt + f) - K_e (cm other + cp self) - C_e(other - <other>) self,
// with M_e = det Mhat, K_e = det sum_pq G_pq Khat_pq and the convection matrix
// C_e = sum_b sum_p T[.][b][.][p] uh[b][p] (uh = det J^-1 (other - <other>) at
// node b).  In the skew-symmetric form C_e is antisymmetric, so only its 15
// upper entries are formed (the strict upper triangle of the 6 x 6 matrix).
//
// Strip: 2 SLOTS - 1 owned cell columns plus one halo column on the left, KS
// owned cell rows plus one halo row below.  The wavefront walks the rows
// upwards; each row runs in four colour phases (lower triangles of the even,
// then odd slot cells, then the upper ones), whose elements share no node, so
// every lane adds its rows to distinct node accumulators.  Accumulators live in
// LDS for the three node lines a cell row touches (line K mod 3); a line is
// final, and written to b, once the rows below and above it are done.  Every
// node therefore sums its elements in the same order (row, then the four
// colours) whatever the strip shape: the result is deterministic, without
// atomics and without an element buffer.  Dirichlet rows take g, pressure rows
// are zero; each P2 node is owned by exactly one wavefront.
struct RhsGrid {
    int nx, ny, nstrips, nseg, nslices, ks;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TO, int M>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) k_rhs_strip(
    const int32_t* __restrict__ cell_el, const int32_t* __restrict__ hs_p2, const int32_t* __restrict__ tri,
    const double* __restrict__ geo, const int32_t* __restrict__ dir_index, const int32_t* __restrict__ p1_of_p2,
    const double* __restrict__ self, const double* __restrict__ other, const double* __restrict__ obar,
    const double* __restrict__ coef, const double* __restrict__ F, const double* __restrict__ G,
    TO* __restrict__ b, RhsGrid gd, int nP2, int J, double inv_dt, int convective) {
    constexpr int SLOTS = 64 / M;
    constexpr int TXO = 2 * SLOTS - 1;          // owned cell columns
    constexpr int NODES = 2 * TXO;              // owned half-step columns
    constexpr int LINE = NODES * 2 * M;         // accumulators of one node line
    // half-step offsets of the local nodes of the lower (0) and upper (1)
    // triangle of a cell, one 4-bit field per node (a register operand, not a table
    // in memory): lower (0,0) (2,0) (2,2) (1,0) (2,1) (1,1), upper (0,0) (2,2)
    // (0,2) (1,1) (1,2) (0,1) as (I, K)
    constexpr unsigned kDI[2] = {0x121220u, 0x011020u};
    constexpr unsigned kDK[2] = {0x110200u, 0x121220u};
    __shared__ double lds[kBlock / 64][3 * LINE];
    __shared__ int topo[kBlock / 64][SLOTS][4][7];   // per phase: the 6 nodes, then the element (-1: none)
    __shared__ int meta[kBlock / 64][3][NODES][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + wv;
    if (w >= (int64_t)gd.nstrips * gd.nseg * gd.nslices) return;    // whole wavefront; no block barrier below
    const int strip = (int)(w % gd.nstrips);
    const int seg = (int)((w / gd.nstrips) % gd.nseg);
    const int slice = (int)(w / ((int64_t)gd.nstrips * gd.nseg));
    const int slot = lane / M, mem = lane % M;
    const int j = slice * M + mem;
    const bool live = j < J;
    const int ci0 = strip * TXO, ck0 = seg * gd.ks;
    const int NXh = 2 * gd.nx + 1;
    const int I0 = 2 * ci0, I1 = min(I0 + NODES, NXh);                  // owned columns [I0, I1)
    const int K0 = 2 * ck0, K1 = min(2 * (ck0 + gd.ks), 2 * gd.ny + 1); // owned lines [K0, K1)
    double* L = lds[wv];
    const double cm = live ? coef[j] : 0.0, cp = live ? coef[J + j] : 0.0;

    auto zero_line = [&](int K) {
        double* ln = L + (K % 3) * LINE;
        for (int q = lane; q < LINE; q += 64) ln[q] = 0.0;
    };
    // node, Dirichlet index and P1 index of the owned nodes of lines 2k .. 2k+2
    // (k the current cell row), fetched once per row
    auto fetch_meta = [&](int k) {
        for (int q = lane; q < 3 * NODES; q += 64) {
            const int l = q / NODES, nd = q % NODES;
            const int I = I0 + nd, K = 2 * k + l;
            int id = -1, di = -1, p1 = -1;
            if (I < I1 && K >= K0 && K < K1) {
                id = hs_p2[(int64_t)K * NXh + I];
                if (id >= 0) {
                    di = dir_index[id];
                    p1 = p1_of_p2[id];
                }
            }
            meta[wv][l][nd][0] = id;
            meta[wv][l][nd][1] = di;
            meta[wv][l][nd][2] = p1;
        }
    };
    auto flush_line = [&](int K, int k) {
        if (K < K0 || K >= K1) return;
        const double* ln = L + (K % 3) * LINE;
        const int l = K - 2 * k;
        for (int q = lane; q < LINE; q += 64) {
            const int mm = q % M, d = (q / M) & 1, nd = q / (2 * M);
            const int jj = slice * M + mm;
            const int id = meta[wv][l][nd][0];
            if (id < 0 || jj >= J) continue;
            const int di = meta[wv][l][nd][1];
            const double v = di >= 0 ? G[(2 * (int64_t)di + d) * J + jj] : ln[q];
            b[(2 * (int64_t)id + d) * J + jj] = (TO)v;
            const int p1 = meta[wv][l][nd][2];
            if (d == 0 && p1 >= 0) b[(2 * (int64_t)nP2 + p1) * J + jj] = (TO)0;
        }
    };

    const int k_first = max(ck0 - 1, 0), k_last = min(ck0 + gd.ks, gd.ny) - 1;
    for (int k = k_first; k <= k_last; ++k) {
        if (k == k_first) zero_line(2 * k);
        zero_line(2 * k + 1);
        zero_line(2 * k + 2);
        wave_sync();
        // the row's four elements of each slot and their nodes, loaded up front by
        // the slot's lanes together into LDS, so that each phase below waits for
        // one round of node-value loads only
        fetch_meta(k);
        for (int q = mem; q < 4 * 7; q += M) {
            const int ph = q / 7, bb = q % 7;
            const int i = ci0 - 1 + 2 * slot + (ph & 1);
            int e = -1;
            if (i >= 0 && i < gd.nx) {
                const int c = cell_el[(int64_t)k * gd.nx + i];
                if (c >= 0) e = c + (ph >> 1);
            }
            topo[wv][slot][ph][bb] = bb == 6 ? e : (e >= 0 ? tri[(int64_t)e * 6 + bb] : 0);
        }
        wave_sync();
#pragma unroll 1
        for (int ph = 0; ph < 4; ++ph) {
            const int up = ph >> 1;
            const int i = ci0 - 1 + 2 * slot + (ph & 1);
            const int e = live ? topo[wv][slot][ph][6] : -1;
            if (e >= 0) {
                // the reference tables are read per element through a constant-
                // address-space pointer the compiler cannot see through, so that it
                // streams them with scalar loads from the scalar cache instead of
                // holding all of them in registers (a generic pointer would turn
                // every table read into a vector memory load; immediate constants
                // spill scalar registers and measured no faster)
                using ConstTables = const __attribute__((address_space(4))) RefTables*;
                ConstTables R = (ConstTables)&c_ref;
                asm volatile("" : "+s"(R));
                const Geo g = load_geo(geo, e);
                double s[6][2], ms[6][2], ks[6][2], uh[6][2];
#pragma unroll
                for (int bb = 0; bb < 6; ++bb) {
                    const int64_t t = topo[wv][slot][ph][bb];
                    double od[2];
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const int64_t idx = (2 * t + d) * J + j;
                        const double sv = self[idx], ov = other[idx];
                        s[bb][d] = sv;
                        ms[bb][d] = sv * inv_dt + (F ? F[idx] : 0.0);
                        ks[bb][d] = cm * ov + cp * sv;
                        od[d] = ov - obar[2 * t + d];
                    }
                    uh[bb][0] = g.det * (g.Ji[0][0] * od[0] + g.Ji[0][1] * od[1]);
                    uh[bb][1] = g.det * (g.Ji[1][0] * od[0] + g.Ji[1][1] * od[1]);
                }
                const double G00 = g.G[0][0], G01 = g.G[0][1], G11 = g.G[1][1];
                double r[6][2];
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    double r0 = 0.0, r1 = 0.0;
#pragma unroll
                    for (int bb = 0; bb < 6; ++bb) {
                        const double m = R->Mhat[a][bb];
                        const double kk = R->Kc[a][bb][0] * G00 + R->Kc[a][bb][1] * G01 + R->Kc[a][bb][2] * G11;
                        r0 = fma(m, ms[bb][0], fma(-kk, ks[bb][0], r0));
                        r1 = fma(m, ms[bb][1], fma(-kk, ks[bb][1], r1));
                    }
                    r[a][0] = g.det * r0;
                    r[a][1] = g.det * r1;
                }
                if (convective) {
#pragma unroll 1
                    for (int a = 0; a < 6; ++a)
#pragma unroll
                        for (int c = 0; c < 6; ++c) {
                            double cf = 0.0;
#pragma unroll
                            for (int bb = 0; bb < 6; ++bb)
                                cf += R->That[a][bb][c][0] * uh[bb][0] + R->That[a][bb][c][1] * uh[bb][1];
                            r[a][0] -= cf * s[c][0];
                            r[a][1] -= cf * s[c][1];
                        }
                } else {
#pragma unroll
                    for (int a = 0; a < 5; ++a)
#pragma unroll
                        for (int c = a + 1; c < 6; ++c) {
                            double cf = 0.0;
#pragma unroll
                            for (int bb = 0; bb < 6; ++bb)
                                cf += R->Shat[a][bb][c][0] * uh[bb][0] + R->Shat[a][bb][c][1] * uh[bb][1];
                            r[a][0] -= cf * s[c][0];
                            r[a][1] -= cf * s[c][1];
                            r[c][0] += cf * s[a][0];
                            r[c][1] += cf * s[a][1];
                        }
                }
                const int ci = 2 * i, ck = 2 * k;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    const int I = ci + (int)(((up ? kDI[1] : kDI[0]) >> (4 * a)) & 15u);
                    const int K = ck + (int)(((up ? kDK[1] : kDK[0]) >> (4 * a)) & 15u);
                    if (I < I0 || I >= I1 || K < K0 || K >= K1) continue;
                    double* acc = L + (K % 3) * LINE + ((I - I0) * 2) * M + mem;
                    acc[0] += r[a][0];
                    acc[M] += r[a][1];
                }
            }
            wave_sync();
        }
        flush_line(2 * k, k);
        flush_line(2 * k + 1, k);
        if (k == k_last) flush_line(2 * k + 2, k);
        wave_sync();
    }
}

// -------------------------------------------------------------- (a3) right-hand sides by node gather
// For meshes without the half-step grid (Scott-Vogelius on the Alfeld
// refinement).  JP lanes per P2 node, the members strided over them.  A lane
// sums, in the node's incidence order (by element), row a of the element
// vector of every element e in which the node is local node a,
//   r = M_e (self/dt + f) - K_e (cm other + cp self) - C_e(other - <other>) self,
// the element arithmetic of the strip kernel, recomputed for each incident
// node instead of accumulated: no element buffer, deterministic.  Dirichlet
// rows take g; pressure rows (units past nP2) are zero.
// WAVE (J > 32): one node per wavefront, JP = 64, so that the node, its
// incidences and each element's local index are uniform and the reference
// tables are read with scalar loads
template <typename TO, bool WAVE>
__global__ void __launch_bounds__(kBlock) k_rhs_nodes(
    const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc, const int32_t* __restrict__ tri,
    const double* __restrict__ geo, const int32_t* __restrict__ dir_index, const double* __restrict__ self,
    const double* __restrict__ other, const double* __restrict__ obar, const double* __restrict__ coef,
    const double* __restrict__ F, const double* __restrict__ G, TO* __restrict__ b, int nP2, int nP1, int J, int JP,
    double inv_dt, int convective) {
    const Lanes L = lanes(JP);
    const int64_t i = WAVE ? (int64_t)__builtin_amdgcn_readfirstlane((int)L.unit) : L.unit;
    if (i >= (int64_t)nP2 + nP1) return;
    if (i >= nP2) {
        for (int j = L.j0; j < J; j += JP) b[(nP2 + i) * J + j] = (TO)0;   // row 2 nP2 + (i - nP2)
        return;
    }
    auto uni = [](int v) { return WAVE ? __builtin_amdgcn_readfirstlane(v) : v; };
    const int di = uni(dir_index[i]);
    const int p0 = uni(inc_ptr[i]), p1 = uni(inc_ptr[i + 1]);
    for (int j = L.j0; j < J; j += JP) {
        if (di >= 0) {
            b[(2 * i) * J + j] = (TO)G[(2 * (int64_t)di) * J + j];
            b[(2 * i + 1) * J + j] = (TO)G[(2 * (int64_t)di + 1) * J + j];
            continue;
        }
        const double cm = coef[j], cp = coef[J + j];
        double acc0 = 0.0, acc1 = 0.0;
        for (int p = p0; p < p1; ++p) {
            const int ea = uni(inc[p]);
            const int e = ea >> 3, a = ea & 7;
            const Geo g = load_geo(geo, e);
            double s[6][2], ms[6][2], ks[6][2], uh[6][2];
#pragma unroll
            for (int bb = 0; bb < 6; ++bb) {
                const int64_t t = tri[(int64_t)e * 6 + bb];
                double od[2];
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int64_t idx = (2 * t + d) * J + j;
                    const double sv = self[idx], ov = other[idx];
                    s[bb][d] = sv;
                    ms[bb][d] = sv * inv_dt + (F ? F[idx] : 0.0);
                    ks[bb][d] = cm * ov + cp * sv;
                    od[d] = ov - obar[2 * t + d];
                }
                uh[bb][0] = g.det * (g.Ji[0][0] * od[0] + g.Ji[0][1] * od[1]);
                uh[bb][1] = g.det * (g.Ji[1][0] * od[0] + g.Ji[1][1] * od[1]);
            }
            const double G00 = g.G[0][0], G01 = g.G[0][1], G11 = g.G[1][1];
            double r0 = 0.0, r1 = 0.0;
#pragma unroll
            for (int bb = 0; bb < 6; ++bb) {
                const double m = c_ref.Mhat[a][bb];
                const double kk = c_ref.Kc[a][bb][0] * G00 + c_ref.Kc[a][bb][1] * G01 + c_ref.Kc[a][bb][2] * G11;
                r0 = fma(m, ms[bb][0], fma(-kk, ks[bb][0], r0));
                r1 = fma(m, ms[bb][1], fma(-kk, ks[bb][1], r1));
            }
            r0 *= g.det;
            r1 *= g.det;
            // convection row a: C[a][c] = sum_b T[a][b][c] . uh[b] (plain) or the
            // antisymmetric part S (skew-symmetric form, zero diagonal)
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                double cf = 0.0;
#pragma unroll
                for (int bb = 0; bb < 6; ++bb)
                    cf += convective ? c_ref.That[a][bb][c][0] * uh[bb][0] + c_ref.That[a][bb][c][1] * uh[bb][1]
                                     : c_ref.Shat[a][bb][c][0] * uh[bb][0] + c_ref.Shat[a][bb][c][1] * uh[bb][1];
                r0 -= cf * s[c][0];
                r1 -= cf * s[c][1];
            }
            acc0 += r0;
            acc1 += r1;
        }
        b[(2 * i) * J + j] = (TO)acc0;
        b[(2 * i + 1) * J + j] = (TO)acc1;
    }
}

// per-node partial of vbar^T M vbar (both components); partial per block
__global__ void __launch_bounds__(kBlock) k_energy(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ valM, const double* __restrict__ vb,
                                                   double* __restrict__ out, int nrows) {
    __shared__ double red[kBlock];
    int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    if (r < nrows) {
        double s0 = 0.0, s1 = 0.0;
        for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
            s0 += valM[p] * vb[2 * col[p]];
            s1 += valM[p] * vb[2 * col[p] + 1];
        }
        acc = vb[2 * r] * s0 + vb[2 * r + 1] * s1;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_mean(const double* z, double* zbar, int64_t rows, int J, hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_mean, dim3(grid_for(rows, JP)), dim3(kBlock), 0, s, z, zbar, rows, J, JP);
    return hipGetLastError();
}

hipError_t launch_eddy_l2(const DevMesh& m, const double* z, const double* zbar, double* l2, int J, hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_eddy_l2, dim3(grid_for(m.n_el, JP)), dim3(kBlock), 0, s, m.tri, z, zbar, l2, m.n_el, J, JP);
    return hipGetLastError();
}

hipError_t launch_assemble_A(const DevMesh& m, const mhd_coeffs& c, const double* zbar, const double* l2, double* elem,
                             double* valA, float* valA32, double* dinvA, float* dinvA32, hipStream_t s) {
    double nu_c = 0.5 * (c.nu_bar + c.num_bar);
    double eddy_c = 2.0 * c.mu * c.dt;
    hipLaunchKernelGGL(k_elem_A, dim3((m.n_el + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.tri, m.geo, zbar, l2,
                       elem, m.n_el, 1.0 / c.dt, nu_c, eddy_c, c.convective);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_A, dim3((m.nP2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.A_rowptr, m.A_col,
                       m.gA_ptr, m.gA_idx, m.dir, elem, valA, valA32, dinvA, dinvA32, m.nP2);
    return hipGetLastError();
}

hipError_t launch_const_assembly(DevMesh& m, double* eb, hipStream_t s) {
    hipLaunchKernelGGL(k_elem_const, dim3((m.n_el + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.geo, eb, m.n_el);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_MK, dim3((m.nP2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.A_rowptr, m.gA_ptr,
                       m.gA_idx, eb, m.valM, m.valK, m.nP2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_B, dim3((m.nP2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.Bt_rowptr, m.gBt_ptr,
                       m.gBt_idx, eb, m.dir, -1, m.valBt, m.valBt32, m.nP2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_B, dim3((m.nP1 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.B_rowptr, m.gB_ptr,
                       m.gB_idx, eb, (const uint8_t*)nullptr, m.pin, m.valB, m.valB32, m.nP1);
    return hipGetLastError();
}

hipError_t launch_member_coefs(const double* nu, const double* nu_m, int J, double* coef, hipStream_t s) {
    hipLaunchKernelGGL(k_member_coefs, dim3(1), dim3(256), 0, s, nu, nu_m, J, coef);
    return hipGetLastError();
}

// one-pass right-hand sides (k_rhs_strip): M members per element slot, ks owned
// cell rows per wavefront
template <typename TO>
hipError_t launch_rhs_strip_t(const DevMesh& m, const mhd_coeffs& c, int J, const double* self_n,
                              const double* other_n, const double* obar, const double* coef, const double* forcing,
                              const double* bc, TO* rhs, hipStream_t s) {
    const int M = J <= 8 ? 8 : 16;
    const int txo = 2 * (64 / M) - 1;
    RhsGrid gd;
    gd.nx = m.nx;
    gd.ny = m.ny;
    gd.ks = 4;
    gd.nstrips = m.nx / txo + 1;
    gd.nseg = m.ny / gd.ks + 1;
    gd.nslices = (J + M - 1) / M;
    const int64_t waves = (int64_t)gd.nstrips * gd.nseg * gd.nslices;
    const dim3 grid((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)));
    if (M == 8)
        hipLaunchKernelGGL((k_rhs_strip<TO, 8>), grid, dim3(kBlock), 0, s, m.cell_el, m.hs_p2, m.tri, m.geo,
                           m.dir_index, m.p1_of_p2, self_n, other_n, obar, coef, forcing, bc, rhs, gd, m.nP2, J,
                           1.0 / c.dt, c.convective);
    else
        hipLaunchKernelGGL((k_rhs_strip<TO, 16>), grid, dim3(kBlock), 0, s, m.cell_el, m.hs_p2, m.tri, m.geo,
                           m.dir_index, m.p1_of_p2, self_n, other_n, obar, coef, forcing, bc, rhs, gd, m.nP2, J,
                           1.0 / c.dt, c.convective);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_rhs_nodes_t(const DevMesh& m, const mhd_coeffs& c, int J, const double* self_n,
                              const double* other_n, const double* obar, const double* coef, const double* forcing,
                              const double* bc, TO* rhs, hipStream_t s) {
    if (J > 32)
        hipLaunchKernelGGL((k_rhs_nodes<TO, true>), dim3(grid_for((int64_t)m.nP2 + m.nP1, 64)), dim3(kBlock), 0, s,
                           m.inc_ptr, m.inc, m.tri, m.geo, m.dir_index, self_n, other_n, obar, coef, forcing, bc, rhs,
                           m.nP2, m.nP1, J, 64, 1.0 / c.dt, c.convective);
    else
        hipLaunchKernelGGL((k_rhs_nodes<TO, false>), dim3(grid_for((int64_t)m.nP2 + m.nP1, pick_jp(J))), dim3(kBlock),
                           0, s, m.inc_ptr, m.inc, m.tri, m.geo, m.dir_index, self_n, other_n, obar, coef, forcing,
                           bc, rhs, m.nP2, m.nP1, J, pick_jp(J), 1.0 / c.dt, c.convective);
    return hipGetLastError();
}

hipError_t launch_rhs_strip(const DevMesh& m, const mhd_coeffs& c, int J, const double* self_n, const double* other_n,
                            const double* obar, const double* coef, const double* forcing, const double* bc,
                            void* rhs, int precision, hipStream_t s) {
    if (sv_mesh(m)) {
        if (precision == MHD_FP32_IR)
            return launch_rhs_nodes_t<float>(m, c, J, self_n, other_n, obar, coef, forcing, bc, (float*)rhs, s);
        return launch_rhs_nodes_t<double>(m, c, J, self_n, other_n, obar, coef, forcing, bc, (double*)rhs, s);
    }
    if (precision == MHD_FP32_IR)
        return launch_rhs_strip_t<float>(m, c, J, self_n, other_n, obar, coef, forcing, bc, (float*)rhs, s);
    return launch_rhs_strip_t<double>(m, c, J, self_n, other_n, obar, coef, forcing, bc, (double*)rhs, s);
}

hipError_t launch_energy_partial(const DevMesh& m, const double* vbar, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3((m.nP2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.A_rowptr, m.A_col,
                       m.valM, vbar, out, m.nP2);
    return hipGetLastError();
}

}  // namespace mhd
