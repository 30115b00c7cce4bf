// Batched solver of libmhd_ens (gfx950): S X = B with one shared saddle-point
// matrix S = [[A (x) I_2, B^T], [B, D_p]] and J member columns (paper,
// Section 1: A [x_1|...|x_J] = [b_1|...|b_J]; Section 4: two Oseen-type
// problems per step).
//
// Method: right-preconditioned restarted GMRES with one Arnoldi process per
// member (per-member Hessenberg matrices and Givens rotations in FP64), one
// SpMM over all J columns per iteration.  Preconditioner (block upper
// triangular): z_p = -S_hat^{-1} r_p with S_hat = B D^{-1} B^T, D the diagonal
// of M/dt + nu_c K (the velocity block without convection), inverted
// approximately by one or two V(2,2)-cycles with damped Jacobi smoothing on a
// Galerkin hierarchy over the nested P1 vertex grids (dense inverse on the
// coarsest level), then z_u = damped Jacobi sweeps on A for r_u - B^T z_p.
// The outer loop is FP64 iterative refinement: r = b - S x in FP64, a GMRES
// cycle in the inner precision (FP32 or FP64) on r, x += d.  A block GMRES
// variant (one Krylov space for all members, with deflation) is an option of
// the adaptive mode.
//
// Every kernel streams member blocks row-major (member index fastest); rows
// are spread over the 8 XCDs in contiguous ranges.  Column reductions go
// through per-block partials and a fixed-order second pass (deterministic).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "device.h"

namespace mhd {

namespace {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 512;    // blocks of the column-reduction kernels

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    int64_t q = G >> 3, r = G & 7, x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

struct Lanes {
    int j0;
    int64_t unit;
};

__device__ __forceinline__ Lanes lanes(int JP) {
    Lanes L;
    int lane = threadIdx.x & 63;
    int wave = threadIdx.x >> 6;
    int rpw = 64 / JP;
    L.j0 = lane % JP;
    int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    L.unit = (blk * (kBlock / 64) + wave) * rpw + lane / JP;
    // one unit per wavefront: make the row index provably uniform so that CSR
    // indices and values are fetched with scalar loads
    if (JP == 64) L.unit = __builtin_amdgcn_readfirstlane((int)L.unit);
    return L;
}

// Fast-path mapping for (n x J) blocks with J a multiple of JT = 32 VEC: one
// wavefront per P2 node and member tile; lane l covers component c = l / 32
// and members jt*JT + (l % 32)*VEC ... + VEC-1, so the node's 2 JT values of
// the tile are read with one VEC-wide load per lane.
struct NodeLanes {
    int c, j;
    int unit;
};

template <int VEC>
__device__ __forceinline__ NodeLanes node_lanes() {
    NodeLanes L;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    L.c = lane >> 5;
    L.j = blockIdx.y * (32 * VEC) + (lane & 31) * VEC;
    int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    L.unit = __builtin_amdgcn_readfirstlane((int)(blk * (kBlock / 64) + wave));
    return L;
}

inline int pick_jp(int J) {
    int p = 1;
    while (p < J && p < 64) p <<= 1;
    return p;
}

inline unsigned grid_for(int64_t units, int JP) {
    int64_t per_block = (kBlock / 64) * (64 / JP);
    return (unsigned)((units + per_block - 1) / per_block);
}

template <typename T>
struct Vals;
template <>
struct Vals<double> {
    static const double* A(const DevShared& s) { return s.transposed ? s.valA_T : s.valA; }
    static const double* dA(const DevShared& s) { return s.dinvA; }
    static const double* B(const DevShared& s) { return s.transposed ? s.mesh->valB_T : s.mesh->valB; }
    static const double* Bt(const DevShared& s) { return s.transposed ? s.mesh->valBt_T : s.mesh->valBt; }
    static const double* dp(const DevMesh& m) { return m.diagp; }
    static const double* csr(const DevCSR<double>& c) { return c.val; }
    static const double* dinv(const DevLevel& l) { return l.dinv; }
    static const double* cinv(const DevLevel& l) { return l.cinv; }
    static int cinv_ld(const DevLevel& l) { return l.n; }
};
template <>
struct Vals<float> {
    static const float* A(const DevShared& s) { return s.transposed ? s.valA_T32 : s.valA32; }
    static const float* dA(const DevShared& s) { return s.dinvA32; }
    static const float* B(const DevShared& s) { return s.transposed ? s.mesh->valB_T32 : s.mesh->valB32; }
    static const float* Bt(const DevShared& s) { return s.transposed ? s.mesh->valBt_T32 : s.mesh->valBt32; }
    static const float* dp(const DevMesh& m) { return m.diagp32; }
    static const float* csr(const DevCSR<double>& c) { return c.val32; }
    static const float* dinv(const DevLevel& l) { return l.dinv32; }
    static const float* cinv(const DevLevel& l) { return l.cinv32; }
    static int cinv_ld(const DevLevel& l) { return l.ld32; }
};

// ------------------------------------------------------------------ saddle-point SpMM
// y = S x (MODE 0) or y = b - S x (MODE 1).  Units: P2 nodes (both velocity
// components) then P1 nodes.  A group of JP lanes handles one unit, lanes over
// members; CSR indices and values are uniform across the group.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_saddle(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                   const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                   const int32_t* __restrict__ Btcol, const T* __restrict__ Btval,
                                                   const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bcol,
                                                   const T* __restrict__ Bval, const T* __restrict__ dp,
                                                   const T* __restrict__ x, const T* __restrict__ bvec,
                                                   T* __restrict__ y, int nP2, int nP1, int J, int JP) {
    Lanes L = lanes(JP);
    const int64_t u = L.unit;
    if (u >= (int64_t)nP2 + nP1) return;
    const T* xp = x + 2 * (int64_t)nP2 * J;
    if (u < nP2) {
        const int32_t a0 = Arp[u], a1 = Arp[u + 1], b0 = Btrp[u], b1 = Btrp[u + 1];
        for (int j = L.j0; j < J; j += JP) {
            T s0 = 0, s1 = 0;
            for (int32_t p = a0; p < a1; ++p) {
                const int64_t k = Acol[p];
                const T a = Aval[p];
                s0 += a * x[(2 * k) * J + j];
                s1 += a * x[(2 * k + 1) * J + j];
            }
            for (int32_t p = b0; p < b1; ++p) {
                const T pv = xp[(int64_t)Btcol[p] * J + j];
                s0 += Btval[2 * p] * pv;
                s1 += Btval[2 * p + 1] * pv;
            }
            if (MODE == 0) {
                y[(2 * u) * J + j] = s0;
                y[(2 * u + 1) * J + j] = s1;
            } else {
                y[(2 * u) * J + j] = bvec[(2 * u) * J + j] - s0;
                y[(2 * u + 1) * J + j] = bvec[(2 * u + 1) * J + j] - s1;
            }
        }
    } else {
        const int64_t k = u - nP2;
        const int32_t q0 = Brp[k], q1 = Brp[k + 1];
        const T d = dp[k];
        const int64_t row = 2 * (int64_t)nP2 + k;
        for (int j = L.j0; j < J; j += JP) {
            T s = d * xp[k * J + j];
            for (int32_t q = q0; q < q1; ++q) {
                const int64_t i = Bcol[q];
                s += Bval[2 * q] * x[(2 * i) * J + j] + Bval[2 * q + 1] * x[(2 * i + 1) * J + j];
            }
            y[row * J + j] = (MODE == 0) ? s : bvec[row * J + j] - s;
        }
    }
}

template <typename T, int VEC>
struct VecT;

template <typename T, int VEC>
__device__ __forceinline__ void vload(T (&v)[VEC], const T* p);
template <typename T, int VEC>
__device__ __forceinline__ void vstore(T* p, const T (&v)[VEC]);

// Fast saddle-point SpMM (see NodeLanes): y = S x (MODE 0) or y = b - S x (MODE 1)
template <typename T, int VEC, int MODE>
__global__ void __launch_bounds__(kBlock) k_saddle_v(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                     const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                     const int32_t* __restrict__ Btcol, const T* __restrict__ Btval,
                                                     const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bcol,
                                                     const T* __restrict__ Bval, const T* __restrict__ dp,
                                                     const T* __restrict__ x, const T* __restrict__ bvec,
                                                     T* __restrict__ y, int nP2, int nP1, int J) {
    const NodeLanes L = node_lanes<VEC>();
    const int u = L.unit;
    if (u >= nP2 + nP1) return;
    const T* xp = x + 2 * (int64_t)nP2 * J;
    T acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = 0;
    if (u < nP2) {
        const int32_t a0 = Arp[u], a1 = Arp[u + 1], b0 = Btrp[u], b1 = Btrp[u + 1];
        const T* xc = x + (int64_t)L.c * J + L.j;
#pragma unroll 4
        for (int32_t p = a0; p < a1; ++p) {
            const int64_t k = Acol[p];
            const T a = Aval[p];
            T v[VEC];
            vload<T, VEC>(v, xc + 2 * k * J);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += a * v[q];
        }
        for (int32_t p = b0; p < b1; ++p) {
            const int64_t m = Btcol[p];
            const T bt = L.c ? Btval[2 * p + 1] : Btval[2 * p];
            T v[VEC];
            vload<T, VEC>(v, xp + m * J + L.j);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += bt * v[q];
        }
        const int64_t o = (2 * (int64_t)u + L.c) * J + L.j;
        if (MODE == 1) {
            T bv[VEC];
            vload<T, VEC>(bv, bvec + o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = bv[q] - acc[q];
        }
        vstore<T, VEC>(y + o, acc);
    } else {
        const int k = u - nP2;
        const int32_t q0 = Brp[k], q1 = Brp[k + 1];
        const T* xc = x + (int64_t)L.c * J + L.j;
#pragma unroll 4
        for (int32_t q = q0; q < q1; ++q) {
            const int64_t i = Bcol[q];
            const T bb = L.c ? Bval[2 * q + 1] : Bval[2 * q];
            T v[VEC];
            vload<T, VEC>(v, xc + 2 * i * J);
#pragma unroll
            for (int r = 0; r < VEC; ++r) acc[r] += bb * v[r];
        }
        // add the two velocity components' contributions (lanes l and l + 32)
#pragma unroll
        for (int r = 0; r < VEC; ++r) acc[r] += __shfl_xor(acc[r], 32, 64);
        if (L.c == 0) {
            const T d = dp[k];
            const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j;
            T v[VEC];
            vload<T, VEC>(v, xp + (int64_t)k * J + L.j);
#pragma unroll
            for (int r = 0; r < VEC; ++r) acc[r] += d * v[r];
            if (MODE == 1) {
                T bv[VEC];
                vload<T, VEC>(bv, bvec + o);
#pragma unroll
                for (int r = 0; r < VEC; ++r) acc[r] = bv[r] - acc[r];
            }
            vstore<T, VEC>(y + o, acc);
        }
    }
}

// Fast velocity-block Jacobi sweeps (see NodeLanes)
// FIRST: t = r_u - B^T z_p ; z = w D^{-1} t
// else:  zo = z + w D^{-1} (t - A z)
template <typename T, int VEC, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_velo_v(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ dinvA,
                                                   const T* __restrict__ in, const T* __restrict__ zp,
                                                   T* __restrict__ t, const T* __restrict__ z, T* __restrict__ zo,
                                                   int nP2, int J, T omega) {
    const NodeLanes L = node_lanes<VEC>();
    const int i = L.unit;
    if (i >= nP2) return;
    const int32_t p0 = rp[i], p1 = rp[i + 1];
    const T dw = omega * dinvA[i];
    const int64_t o = (2 * (int64_t)i + L.c) * J + L.j;
    T acc[VEC];
    if (FIRST) {
        vload<T, VEC>(acc, in + o);                       // r_u
#pragma unroll 4
        for (int32_t p = p0; p < p1; ++p) {
            const int64_t m = col[p];
            const T bt = L.c ? val[2 * p + 1] : val[2 * p];
            T v[VEC];
            vload<T, VEC>(v, zp + m * J + L.j);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] -= bt * v[q];
        }
        vstore<T, VEC>(t + o, acc);
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] *= dw;
        vstore<T, VEC>(zo + o, acc);
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = 0;
        const T* zc = z + (int64_t)L.c * J + L.j;
#pragma unroll 4
        for (int32_t p = p0; p < p1; ++p) {
            const int64_t k = col[p];
            const T a = val[p];
            T v[VEC];
            vload<T, VEC>(v, zc + 2 * k * J);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += a * v[q];
        }
        T tv[VEC], zv[VEC];
        vload<T, VEC>(tv, t + o);
        vload<T, VEC>(zv, z + o);
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = zv[q] + dw * (tv[q] - acc[q]);
        vstore<T, VEC>(zo + o, acc);
    }
}

// ------------------------------------------------------------------ batched-gather node-row kernels
// Same lane layout as NodeLanes, but a wavefront handles G consecutive units
// and gathers a row in batches: lane t first loads the row's t-th column index
// and value (one coalesced load for the whole row), then the column indices are
// broadcast with v_readlane so that 4 or 8 member-row loads of x are in flight
// before the first multiply-add.  Rows are padded to the batch width with a
// valid column and a zero value; a row may hold at most kMaxRowBatched entries.
constexpr int kMaxRowBatched = 56;

__device__ __forceinline__ float lane_bcast(float v, int t) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), t));
}
__device__ __forceinline__ double lane_bcast(double v, int t) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), t);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), t);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ int rl(int v, int i) { return __builtin_amdgcn_readlane(v, i); }

// One row's entries spread over the lanes: lane t < cnt holds entry t.  With
// PAIR the row has two values per entry (one per velocity component).
template <typename T, bool PAIR>
struct RowLanes {
    int cnt;
    int col;
    T v0, v1;
};

template <typename T, bool PAIR>
__device__ __forceinline__ RowLanes<T, PAIR> row_lanes(const int32_t* __restrict__ col, const T* __restrict__ val,
                                                       int32_t p0, int32_t p1, int pad_col) {
    RowLanes<T, PAIR> R;
    const int lane = threadIdx.x & 63;
    R.cnt = p1 - p0;
    R.col = pad_col;
    R.v0 = 0;
    R.v1 = 0;
    if (lane < R.cnt) {
        R.col = col[p0 + lane];
        if (PAIR) {
            R.v0 = val[2 * (p0 + lane)];
            R.v1 = val[2 * (p0 + lane) + 1];
        } else {
            R.v0 = val[p0 + lane];
        }
    }
    return R;
}

// acc[q] += sum over entries t in [t0, t0 + NB) of a_t * xb[col_t * cstride + q]
// (NEG: acc[q] -= ..., with the same fused multiply-adds as a sequential loop)
template <typename T, int VEC, int NB, bool PAIR, bool NEG>
__device__ __forceinline__ void gather_batch(const RowLanes<T, PAIR>& R, int t0, int c, const T* __restrict__ xb,
                                             int64_t cstride, T (&acc)[VEC]) {
    T v[NB][VEC];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int64_t k = __builtin_amdgcn_readlane(R.col, t0 + i);
        vload<T, VEC>(v[i], xb + k * cstride);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        T a;
        if (PAIR) {
            const T a0 = lane_bcast(R.v0, t0 + i), a1 = lane_bcast(R.v1, t0 + i);
            a = c ? a1 : a0;
        } else {
            a = lane_bcast(R.v0, t0 + i);
        }
        if (NEG) a = -a;
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] += a * v[i][q];
    }
}

template <typename T, int VEC, bool PAIR, bool NEG = false>
__device__ __forceinline__ void gather_row(const RowLanes<T, PAIR>& R, int c, const T* __restrict__ xb, int64_t cstride,
                                           T (&acc)[VEC]) {
    int t = 0;
    for (; t + 8 <= R.cnt; t += 8) gather_batch<T, VEC, 8, PAIR, NEG>(R, t, c, xb, cstride, acc);
    const int r = R.cnt - t;
    if (r > 4)
        gather_batch<T, VEC, 8, PAIR, NEG>(R, t, c, xb, cstride, acc);
    else if (r > 0)
        gather_batch<T, VEC, 4, PAIR, NEG>(R, t, c, xb, cstride, acc);
}

struct GroupLanes {
    int c, j;
    int u0;   // first unit of this wavefront (uniform)
};

template <int VEC, int G>
__device__ __forceinline__ GroupLanes group_lanes() {
    GroupLanes L;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    L.c = lane >> 5;
    L.j = blockIdx.y * (32 * VEC) + (lane & 31) * VEC;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    L.u0 = __builtin_amdgcn_readfirstlane((int)((blk * (kBlock / 64) + wave) * G));
    return L;
}

// y = S x (MODE 0) or y = b - S x (MODE 1), G units per wavefront
template <typename T, int VEC, int MODE, int G>
__global__ void __launch_bounds__(kBlock) k_saddle_g(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                     const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                     const int32_t* __restrict__ Btcol, const T* __restrict__ Btval,
                                                     const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bcol,
                                                     const T* __restrict__ Bval, const T* __restrict__ dp,
                                                     const T* __restrict__ x, const T* __restrict__ bvec,
                                                     T* __restrict__ y, int nP2, int nP1, int J,
                                                     const int32_t* __restrict__ sched) {
    GroupLanes L = group_lanes<VEC, G>();
    int uend = nP2 + nP1;
    if (sched) {   // wave order as in pair_lanes (P1 wavefronts interleaved with the P2 ones)
        const int w = L.u0 / G;
        if (w >= (nP2 + G - 1) / G + (nP1 + G - 1) / G) return;
        const int d = sched[w];
        L.u0 = d >= 0 ? d : nP2 + (-d - 1);
        uend = d >= 0 ? nP2 : nP2 + nP1;
    }
    const T* xp = x + 2 * (int64_t)nP2 * J;
    const T* xc = x + (int64_t)L.c * J + L.j;
    for (int g = 0; g < G; ++g) {
        const int u = L.u0 + g;
        if (u >= uend) return;
        T acc[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = 0;
        if (u < nP2) {
            const RowLanes<T, false> RA = row_lanes<T, false>(Acol, Aval, Arp[u], Arp[u + 1], u);
            const RowLanes<T, true> RB = row_lanes<T, true>(Btcol, Btval, Btrp[u], Btrp[u + 1], 0);
            gather_row<T, VEC, false>(RA, L.c, xc, 2 * (int64_t)J, acc);
            gather_row<T, VEC, true>(RB, L.c, xp + L.j, J, acc);
            const int64_t o = (2 * (int64_t)u + L.c) * J + L.j;
            if (MODE == 1) {
                T bv[VEC];
                vload<T, VEC>(bv, bvec + o);
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] = bv[q] - acc[q];
            }
            vstore<T, VEC>(y + o, acc);
        } else {
            const int k = u - nP2;
            const RowLanes<T, true> RB = row_lanes<T, true>(Bcol, Bval, Brp[k], Brp[k + 1], 0);
            gather_row<T, VEC, true>(RB, L.c, xc, 2 * (int64_t)J, acc);
            // add the two velocity components' contributions (lanes l and l + 32)
#pragma unroll
            for (int r = 0; r < VEC; ++r) acc[r] += __shfl_xor(acc[r], 32, 64);
            if (L.c == 0) {
                const T d = dp[k];
                const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j;
                T v[VEC];
                vload<T, VEC>(v, xp + (int64_t)k * J + L.j);
#pragma unroll
                for (int r = 0; r < VEC; ++r) acc[r] += d * v[r];
                if (MODE == 1) {
                    T bv[VEC];
                    vload<T, VEC>(bv, bvec + o);
#pragma unroll
                    for (int r = 0; r < VEC; ++r) acc[r] = bv[r] - acc[r];
                }
                vstore<T, VEC>(y + o, acc);
            }
        }
    }
}

// Velocity-block Jacobi sweeps, G nodes per wavefront (operations as k_velo_v)
template <typename T, int VEC, bool FIRST, int G>
__global__ void __launch_bounds__(kBlock) k_velo_g(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ dinvA,
                                                   const T* __restrict__ in, const T* __restrict__ zp,
                                                   T* __restrict__ t, const T* __restrict__ z, T* __restrict__ zo,
                                                   int nP2, int J, T omega) {
    const GroupLanes L = group_lanes<VEC, G>();
    for (int g = 0; g < G; ++g) {
        const int i = L.u0 + g;
        if (i >= nP2) return;
        const T dw = omega * dinvA[i];
        const int64_t o = (2 * (int64_t)i + L.c) * J + L.j;
        T acc[VEC];
        if (FIRST) {
            const RowLanes<T, true> RB = row_lanes<T, true>(col, val, rp[i], rp[i + 1], 0);
            vload<T, VEC>(acc, in + o);   // r_u
            gather_row<T, VEC, true, true>(RB, L.c, zp + L.j, J, acc);
            vstore<T, VEC>(t + o, acc);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] *= dw;
            vstore<T, VEC>(zo + o, acc);
        } else {
            const RowLanes<T, false> RA = row_lanes<T, false>(col, val, rp[i], rp[i + 1], i);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = 0;
            gather_row<T, VEC, false>(RA, L.c, z + (int64_t)L.c * J + L.j, 2 * (int64_t)J, acc);
            T tv[VEC], zv[VEC];
            vload<T, VEC>(tv, t + o);
            vload<T, VEC>(zv, z + o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = zv[q] + dw * (tv[q] - acc[q]);
            vstore<T, VEC>(zo + o, acc);
        }
    }
}

// ------------------------------------------------------------------ pipelined gather kernels
// Gather kernels with deep memory-level parallelism: a wavefront owns G
// consecutive units; the CSR bounds of all G rows come in with one load per
// lane, the next row's column indices and values are loaded while the current
// row is computed, and all member-row loads of a row (up to kDeepA entries of
// A or B, kDeepBt of B^T, padded to batches of 8) are in flight before the
// first multiply-add.  Lane layout as NodeLanes.
constexpr int kDeepA = 24;
constexpr int kDeepBt = 8;

template <typename T, bool PAIR>
__device__ __forceinline__ T entry_value(const RowLanes<T, PAIR>& R, int t, int c) {
    if (PAIR) {
        const T a0 = lane_bcast(R.v0, t), a1 = lane_bcast(R.v1, t);
        return c ? a1 : a0;
    }
    return lane_bcast(R.v0, t);
}

// acc[q] += sum_t a_t xb[col_t cstride + q] over a row of at most NBAT batches
// of 8 entries: every load is issued before the first multiply-add
template <typename T, int VEC, int NBAT, bool PAIR, bool NEG>
__device__ __forceinline__ void deep_row(const RowLanes<T, PAIR>& R, int c, const T* __restrict__ xb, int64_t cstride,
                                         T (&acc)[VEC]) {
    const int nb = (R.cnt + 7) >> 3;
    T v[NBAT][8][VEC];
#pragma unroll
    for (int b = 0; b < NBAT; ++b)
        if (b < nb) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t k = __builtin_amdgcn_readlane(R.col, 8 * b + i);
                vload<T, VEC>(v[b][i], xb + k * cstride);
            }
        }
#pragma unroll
    for (int b = 0; b < NBAT; ++b)
        if (b < nb) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                T a = entry_value<T, PAIR>(R, 8 * b + i, c);
                if (NEG) a = -a;
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] += a * v[b][i][q];
            }
        }
}

template <typename T>
struct DeepRows {
    RowLanes<T, false> A;   // A row of a P2 unit
    RowLanes<T, true> B;    // B^T row of a P2 unit, or B row of a P1 unit
};

// y = S x (MODE 0) or y = b - S x (MODE 1), G units per wavefront
template <typename T, int VEC, int MODE, int G>
__global__ void __launch_bounds__(kBlock) k_saddle_p(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                     const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                     const int32_t* __restrict__ Btcol, const T* __restrict__ Btval,
                                                     const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bcol,
                                                     const T* __restrict__ Bval, const T* __restrict__ dp,
                                                     const T* __restrict__ x, const T* __restrict__ bvec,
                                                     T* __restrict__ y, int nP2, int nP1, int J) {
    const GroupLanes L = group_lanes<VEC, G>();
    const int n = min(G, nP2 + nP1 - L.u0);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63;
    int m0 = 0, m1 = 0, m2 = 0, m3 = 0;   // CSR bounds of unit u0 + lane
    if (lane < n) {
        const int u = L.u0 + lane;
        if (u < nP2) {
            m0 = Arp[u];
            m1 = Arp[u + 1];
            m2 = Btrp[u];
            m3 = Btrp[u + 1];
        } else {
            m2 = Brp[u - nP2];
            m3 = Brp[u - nP2 + 1];
        }
    }
    auto load = [&](int g) {
        DeepRows<T> R;
        const int u = L.u0 + g;
        if (u < nP2) {
            R.A = row_lanes<T, false>(Acol, Aval, rl(m0, g), rl(m1, g), u);
            R.B = row_lanes<T, true>(Btcol, Btval, rl(m2, g), rl(m3, g), 0);
        } else {
            R.A.cnt = 0;
            R.A.col = 0;
            R.A.v0 = R.A.v1 = 0;
            R.B = row_lanes<T, true>(Bcol, Bval, rl(m2, g), rl(m3, g), 0);
        }
        return R;
    };
    const T* xp = x + 2 * (int64_t)nP2 * J;
    const T* xc = x + (int64_t)L.c * J + L.j;
    DeepRows<T> cur = load(0);
    for (int g = 0; g < n; ++g) {
        DeepRows<T> nxt = cur;
        if (g + 1 < n) nxt = load(g + 1);
        const int u = L.u0 + g;
        T acc[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = 0;
        if (u < nP2) {
            deep_row<T, VEC, kDeepA / 8, false, false>(cur.A, L.c, xc, 2 * (int64_t)J, acc);
            deep_row<T, VEC, kDeepBt / 8, true, false>(cur.B, L.c, xp + L.j, J, acc);
            const int64_t o = (2 * (int64_t)u + L.c) * J + L.j;
            if (MODE == 1) {
                T bv[VEC];
                vload<T, VEC>(bv, bvec + o);
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc[q] = bv[q] - acc[q];
            }
            vstore<T, VEC>(y + o, acc);
        } else {
            const int k = u - nP2;
            deep_row<T, VEC, kDeepA / 8, true, false>(cur.B, L.c, xc, 2 * (int64_t)J, acc);
#pragma unroll
            for (int r = 0; r < VEC; ++r) acc[r] += __shfl_xor(acc[r], 32, 64);
            if (L.c == 0) {
                const T d = dp[k];
                const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j;
                T v[VEC];
                vload<T, VEC>(v, xp + (int64_t)k * J + L.j);
#pragma unroll
                for (int r = 0; r < VEC; ++r) acc[r] += d * v[r];
                if (MODE == 1) {
                    T bv[VEC];
                    vload<T, VEC>(bv, bvec + o);
#pragma unroll
                    for (int r = 0; r < VEC; ++r) acc[r] = bv[r] - acc[r];
                }
                vstore<T, VEC>(y + o, acc);
            }
        }
        cur = nxt;
    }
}

// velocity-block Jacobi sweeps, pipelined (operations as k_velo_v)
template <typename T, int VEC, bool FIRST, int G>
__global__ void __launch_bounds__(kBlock) k_velo_p(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ dinvA,
                                                   const T* __restrict__ in, const T* __restrict__ zp,
                                                   T* __restrict__ t, const T* __restrict__ z, T* __restrict__ zo,
                                                   int nP2, int J, T omega) {
    const GroupLanes L = group_lanes<VEC, G>();
    const int n = min(G, nP2 - L.u0);
    if (n <= 0) return;
    const int lane = threadIdx.x & 63;
    int m0 = 0, m1 = 0;
    if (lane < n) {
        m0 = rp[L.u0 + lane];
        m1 = rp[L.u0 + lane + 1];
    }
    auto load = [&](int g) {
        return row_lanes<T, FIRST>(col, val, rl(m0, g), rl(m1, g), FIRST ? 0 : L.u0 + g);
    };
    RowLanes<T, FIRST> cur = load(0);
    for (int g = 0; g < n; ++g) {
        RowLanes<T, FIRST> nxt = cur;
        if (g + 1 < n) nxt = load(g + 1);
        const int i = L.u0 + g;
        const T dw = omega * dinvA[i];
        const int64_t o = (2 * (int64_t)i + L.c) * J + L.j;
        T acc[VEC];
        if constexpr (FIRST) {
            vload<T, VEC>(acc, in + o);   // r_u
            deep_row<T, VEC, kDeepBt / 8, true, true>(cur, L.c, zp + L.j, J, acc);
            vstore<T, VEC>(t + o, acc);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] *= dw;
            vstore<T, VEC>(zo + o, acc);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = 0;
            deep_row<T, VEC, kDeepA / 8, false, false>(cur, L.c, z + (int64_t)L.c * J + L.j, 2 * (int64_t)J, acc);
            T tv[VEC], zv[VEC];
            vload<T, VEC>(tv, t + o);
            vload<T, VEC>(zv, z + o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = zv[q] + dw * (tv[q] - acc[q]);
            vstore<T, VEC>(zo + o, acc);
        }
        cur = nxt;
    }
}

// ------------------------------------------------------------------ paired-row gather kernels
// Two rows per wavefront at a time: lanes 0-31 compute one row and lanes 32-63
// another, each half covering both velocity components of MJ = 16 V members
// with 16-byte loads (V = 16 / sizeof(T) members per lane), so every load
// instruction fetches two member rows of x.  A wavefront owns G consecutive
// units of one kind (P2 or P1) and pairs unit g with unit g + G/2.  Within a
// half, lane h covers component h / 16 and members (h % 16) V ... + V - 1.
// Lane h of a half first turns the row's h-th entry into a byte offset of the
// member row it reads; per entry the offset and value are broadcast within the
// half (ds_bpermute) and the load is a buffer load with that offset.  Rows are
// padded with zero values to the longer row of the pair; entries are consumed
// in CSR order, so the arithmetic matches the other kernels.
constexpr int kPairRow = 32;   // entries of a row the paired kernels take per chunk

struct PairLanes {
    int half, c, j;
    int u0, uend;   // units [u0, u0 + G) of this wavefront, clipped to uend (uniform)
};

// sched (optional): wave order; entry >= 0 is a wavefront of P2 units starting
// at that unit, entry < 0 one of P1 units starting at nP2 + (-entry - 1)
template <int V, int G>
__device__ __forceinline__ PairLanes pair_lanes(int nP2, int nP1, int wP2, const int32_t* __restrict__ sched = nullptr) {
    PairLanes L;
    const int lane = threadIdx.x & 63;
    L.half = lane >> 5;
    const int h = lane & 31;
    L.c = h >> 4;
    L.j = blockIdx.y * (16 * V) + (h & 15) * V;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane((int)(blk * (kBlock / 64) + (threadIdx.x >> 6)));
    if (sched) {
        const int nw = (nP2 + G - 1) / G + (nP1 + G - 1) / G;
        const int d = w < nw ? sched[w] : -(nP1 + 1);   // past the schedule: an empty P1 wavefront
        if (d >= 0) {
            L.u0 = d;
            L.uend = nP2;
        } else {
            L.u0 = nP2 + (-d - 1);
            L.uend = nP2 + nP1;
        }
    } else if (w < wP2) {
        L.u0 = w * G;
        L.uend = nP2;
    } else {
        L.u0 = nP2 + (w - wP2) * G;
        L.uend = nP2 + nP1;
    }
    return L;
}

template <typename T>
__device__ __forceinline__ T half_bcast(T v, int src) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
    } else {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffLL));
        const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
}

// ds_bpermute with a byte address (lane * 4)
template <typename T>
__device__ __forceinline__ T bperm_addr(T v, int addr) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
    } else {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
        const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
}

// lane h of a half holds entry h of its half's row: byte offset of the member
// row the entry reads (column * row_bytes + base_bytes; entries past the row
// read the first member row with a zero value) and the value(s)
template <typename T, bool PAIR>
struct HalfRow {
    int cnt;         // entries of this lane's row
    unsigned off;
    T v0, v1;
};

template <typename T, bool PAIR>
__device__ __forceinline__ HalfRow<T, PAIR> half_row(const int32_t* __restrict__ col, const T* __restrict__ val,
                                                     int32_t p0, int32_t p1, unsigned row_bytes,
                                                     unsigned base_bytes) {
    HalfRow<T, PAIR> R;
    const int h = threadIdx.x & 31;
    R.cnt = p1 - p0;
    R.off = base_bytes;
    R.v0 = 0;
    R.v1 = 0;
    if (h < R.cnt) {
        R.off = (unsigned)col[p0 + h] * row_bytes + base_bytes;
        if (PAIR) {
            R.v0 = val[2 * (p0 + h)];
            R.v1 = val[2 * (p0 + h) + 1];
        } else {
            R.v0 = val[p0 + h];
        }
    }
    return R;
}

// a buffer resource over `bytes` bytes from p (loads past the end return 0)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T, int V>
__device__ __forceinline__ void bload(T (&v)[V], __amdgpu_buffer_rsrc_t r, unsigned off) {
    static_assert(sizeof(T) * V == 16, "16-byte member loads");
    auto w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    __builtin_memcpy(v, &w, 16);
}

// acc[q] += sum_t a_t x[off_t + lane_off + q] over entries t0 ... t0 + B - 1
// (B loads in flight)
template <typename T, int V, bool PAIR, bool NEG, int B>
__device__ __forceinline__ void pair_batch(const HalfRow<T, PAIR>& R, int t0, int hb, int c,
                                           __amdgpu_buffer_rsrc_t xr, unsigned lane_off, T (&acc)[V]) {
    T v[B][V];
    T a[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int addr = hb + ((t0 + i) << 2);
        const unsigned off = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)R.off);
        bload<T, V>(v[i], xr, off + lane_off);
        if (PAIR) {
            const T a0 = bperm_addr(R.v0, addr), a1 = bperm_addr(R.v1, addr);
            a[i] = c ? a1 : a0;
        } else {
            a[i] = bperm_addr(R.v0, addr);
        }
        if (NEG) a[i] = -a[i];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
        for (int q = 0; q < V; ++q) acc[q] += a[i] * v[i][q];
    }
}

// Runs batch(std::integral_constant<int, B>, t0) over entries 0 ... n - 1 in
// order: batches of 8 loads, then the remainder r < 8 as 8 (r = 7), 4 + 2 or
// 4 + 1 (r = 6, 5), 4 (r = 3, 4), 2 or 1; entries past the row add zero
template <typename F>
__device__ __forceinline__ void pair_batches(int n, F&& batch) {
    int t = 0;
    for (; t + 8 <= n; t += 8) batch(std::integral_constant<int, 8>{}, t);
    int r = n - t;
    if (r == 7) {
        batch(std::integral_constant<int, 8>{}, t);
        return;
    }
    if (r >= 3) {
        batch(std::integral_constant<int, 4>{}, t);
        t += 4;
        r -= 4;
    }
    if (r == 2) batch(std::integral_constant<int, 2>{}, t);
    if (r == 1) batch(std::integral_constant<int, 1>{}, t);
}

// acc[q] += sum_t a_t x[off_t + lane_off + q] for this lane's row; n = entries
// of the longer row of the pair (uniform, <= kPairRow), in entry order
template <typename T, int V, bool PAIR, bool NEG>
__device__ __forceinline__ void pair_row(const HalfRow<T, PAIR>& R, int n, int half, int c,
                                         __amdgpu_buffer_rsrc_t xr, unsigned lane_off, T (&acc)[V]) {
    const int hb = half << 7;   // byte address of lane 32 half
    pair_batches(n, [&](auto nb, int t0) {
        pair_batch<T, V, PAIR, NEG, decltype(nb)::value>(R, t0, hb, c, xr, lane_off, acc);
    });
}

// pair_row over rows of any length: entries in chunks of kPairRow (one chunk,
// the same operations, for rows of at most kPairRow entries)
template <typename T, int V, bool PAIR, bool NEG>
__device__ __forceinline__ void pair_row_long(const int32_t* __restrict__ col, const T* __restrict__ val, int32_t p0,
                                              int32_t p1, unsigned row_bytes, unsigned base_bytes, int half, int c,
                                              __amdgpu_buffer_rsrc_t xr, unsigned lane_off, T (&acc)[V]) {
    const int cnt = p1 - p0;
    const int n = max(__builtin_amdgcn_readlane(cnt, 0), __builtin_amdgcn_readlane(cnt, 32));
    for (int b = 0; b < n; b += kPairRow) {
        const HalfRow<T, PAIR> R = half_row<T, PAIR>(col, val, p0 + b, p1, row_bytes, base_bytes);
        pair_row<T, V, PAIR, NEG>(R, min(kPairRow, n - b), half, c, xr, lane_off, acc);
    }
}

// y = S x (MODE 0) or y = b - S x (MODE 1)
template <typename T, int MODE, int G>
__global__ void __launch_bounds__(kBlock) k_saddle_h(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                     const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                     const int32_t* __restrict__ Btcol, const T* __restrict__ Btval,
                                                     const int32_t* __restrict__ Brp, const int32_t* __restrict__ Bcol,
                                                     const T* __restrict__ Bval, const T* __restrict__ dp,
                                                     const T* __restrict__ x, const T* __restrict__ bvec,
                                                     T* __restrict__ y, int nP2, int nP1, int J, int wP2,
                                                     const int32_t* __restrict__ sched) {
    constexpr int V = 16 / (int)sizeof(T);
    const PairLanes L = pair_lanes<V, G>(nP2, nP1, wP2, sched);
    const unsigned W = sizeof(T);
    const __amdgpu_buffer_rsrc_t xr = make_rsrc(x, (unsigned)((2 * (int64_t)nP2 + nP1) * J * W));
    const unsigned vrow = 2u * J * W;                      // bytes per velocity node (both components)
    const unsigned pbase = 2u * (unsigned)nP2 * J * W;     // start of the pressure block
    const unsigned lane_v = ((unsigned)L.c * J + L.j) * W, lane_p = (unsigned)L.j * W;
    for (int s = 0; s < G / 2; ++s) {
        const int ua = L.u0 + s, ub = L.u0 + s + G / 2;
        if (ua >= L.uend) return;
        const bool has_b = ub < L.uend;
        const int u = (L.half && has_b) ? ub : ua;   // a lone row is computed twice, stored once
        T acc[V];
#pragma unroll
        for (int q = 0; q < V; ++q) acc[q] = 0;
        if (u < nP2) {
            pair_row_long<T, V, false, false>(Acol, Aval, Arp[u], Arp[u + 1], vrow, 0, L.half, L.c, xr, lane_v, acc);
            pair_row_long<T, V, true, false>(Btcol, Btval, Btrp[u], Btrp[u + 1], J * W, pbase, L.half, L.c, xr,
                                             lane_p, acc);
            const int64_t o = (2 * (int64_t)u + L.c) * J + L.j;
            if (MODE == 1) {
                T bv[V];
                vload<T, V>(bv, bvec + o);
#pragma unroll
                for (int q = 0; q < V; ++q) acc[q] = bv[q] - acc[q];
            }
            if (!L.half || has_b) vstore<T, V>(y + o, acc);
        } else {
            const int k = u - nP2;
            pair_row_long<T, V, true, false>(Bcol, Bval, Brp[k], Brp[k + 1], vrow, 0, L.half, L.c, xr, lane_v, acc);
#pragma unroll
            for (int r = 0; r < V; ++r) acc[r] += __shfl_xor(acc[r], 16, 64);   // the two components
            if (L.c == 0 && (!L.half || has_b)) {
                const T d = dp[k];
                const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j;
                T v[V];
                vload<T, V>(v, x + (2 * (int64_t)nP2 + k) * J + L.j);
#pragma unroll
                for (int r = 0; r < V; ++r) acc[r] += d * v[r];
                if (MODE == 1) {
                    T bv[V];
                    vload<T, V>(bv, bvec + o);
#pragma unroll
                    for (int r = 0; r < V; ++r) acc[r] = bv[r] - acc[r];
                }
                vstore<T, V>(y + o, acc);
            }
        }
    }
}

// velocity-block Jacobi, paired rows (operations as k_velo_v); units are P2 only
template <typename T, bool FIRST, int G>
__global__ void __launch_bounds__(kBlock) k_velo_h(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ dinvA,
                                                   const T* __restrict__ in, const T* __restrict__ zp,
                                                   T* __restrict__ t, const T* __restrict__ z, T* __restrict__ zo,
                                                   int nP2, int J, T omega) {
    constexpr int V = 16 / (int)sizeof(T);
    const PairLanes L = pair_lanes<V, G>(nP2, 0, 1 << 30);
    const unsigned W = sizeof(T);
    // FIRST gathers from the pressure block zp (nP1 rows of J), the sweeps from z
    const __amdgpu_buffer_rsrc_t xr =
        FIRST ? make_rsrc(zp, 0x7fffffffu) : make_rsrc(z, (unsigned)(2 * (int64_t)nP2 * J * W));
    const unsigned lane_off = FIRST ? (unsigned)L.j * W : ((unsigned)L.c * J + L.j) * W;
    const unsigned row_bytes = FIRST ? J * W : 2u * J * W;
    for (int s = 0; s < G / 2; ++s) {
        const int ua = L.u0 + s, ub = L.u0 + s + G / 2;
        if (ua >= L.uend) return;
        const bool has_b = ub < L.uend;
        const int i = (L.half && has_b) ? ub : ua;
        const bool store = !L.half || has_b;
        const T dw = omega * dinvA[i];
        const int64_t o = (2 * (int64_t)i + L.c) * J + L.j;
        T acc[V];
        if constexpr (FIRST) {
            vload<T, V>(acc, in + o);   // r_u
            pair_row_long<T, V, true, true>(col, val, rp[i], rp[i + 1], row_bytes, 0, L.half, L.c, xr, lane_off, acc);
            if (store) vstore<T, V>(t + o, acc);
#pragma unroll
            for (int q = 0; q < V; ++q) acc[q] *= dw;
            if (store && zo) vstore<T, V>(zo + o, acc);   // no zo: the next kernel forms w D^-1 t itself
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) acc[q] = 0;
            pair_row_long<T, V, false, false>(col, val, rp[i], rp[i + 1], row_bytes, 0, L.half, L.c, xr, lane_off,
                                              acc);
            T tv[V], zv[V];
            vload<T, V>(tv, t + o);
            vload<T, V>(zv, z + o);
#pragma unroll
            for (int q = 0; q < V; ++q) acc[q] = zv[q] + dw * (tv[q] - acc[q]);
            if (store) vstore<T, V>(zo + o, acc);
        }
    }
}

// a * b rounded on its own: the product carries no contraction flag, so it is
// never fused into a neighbouring add
template <typename T>
__device__ __forceinline__ T mul_rn(T a, T b) {
#pragma clang fp contract(off)
    return a * b;
}

// acc[q] += sum_t a_t (x[off_t + lane_off + q] s_t) with a per-entry scale s_t
// (held in R.v1 by the entry's lane), the operations of forming the scaled
// vector first and then the product
template <typename T, int V>
__device__ __forceinline__ void pair_row_scaled(const HalfRow<T, false>& R, int n, int half,
                                                __amdgpu_buffer_rsrc_t xr, unsigned lane_off, T (&acc)[V]) {
    const int hb = half << 7;
    auto batch = [&](auto nb, int t0) {
        constexpr int B = decltype(nb)::value;
        T v[B][V];
        T a[B], sc[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int addr = hb + ((t0 + i) << 2);
            const unsigned off = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)R.off);
            bload<T, V>(v[i], xr, off + lane_off);
            a[i] = bperm_addr(R.v0, addr);
            sc[i] = bperm_addr(R.v1, addr);
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const T zq = mul_rn(v[i][q], sc[i]);
                acc[q] += a[i] * zq;
            }
        }
    };
    pair_batches(n, batch);
}

// The second velocity Jacobi sweep straight from t, paired rows: with
// z1 = w D^-1 t formed on the fly for the row and its neighbours,
// zo = z1 + w D^-1 (t - A z1), the same operations as the first sweep's z1
// store followed by k_velo_h (so the first sweep need not store z1).
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_velo_h2(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    const T* __restrict__ val, const T* __restrict__ dinvA,
                                                    const T* __restrict__ t, T* __restrict__ zo, int nP2, int J,
                                                    T omega) {
    constexpr int V = 16 / (int)sizeof(T);
    const PairLanes L = pair_lanes<V, G>(nP2, 0, 1 << 30);
    const unsigned W = sizeof(T);
    const __amdgpu_buffer_rsrc_t tr = make_rsrc(t, (unsigned)(2 * (int64_t)nP2 * J * W));
    const unsigned lane_off = ((unsigned)L.c * J + L.j) * W;
    for (int s = 0; s < G / 2; ++s) {
        const int ua = L.u0 + s, ub = L.u0 + s + G / 2;
        if (ua >= L.uend) return;
        const bool has_b = ub < L.uend;
        const int i = (L.half && has_b) ? ub : ua;
        const bool store = !L.half || has_b;
        const T dw = omega * dinvA[i];
        const int64_t o = (2 * (int64_t)i + L.c) * J + L.j;
        T acc[V], tv[V];
        vload<T, V>(tv, t + o);
#pragma unroll
        for (int q = 0; q < V; ++q) acc[q] = 0;
        const int32_t p0 = rp[i], p1 = rp[i + 1];
        const int cnt = p1 - p0;
        const int n = max(__builtin_amdgcn_readlane(cnt, 0), __builtin_amdgcn_readlane(cnt, 32));
        for (int b = 0; b < n; b += kPairRow) {   // rows longer than kPairRow in chunks
            HalfRow<T, false> R = half_row<T, false>(col, val, p0 + b, p1, 2u * J * W, 0);
            {   // the entry's scale w D^-1 of its column, in the unused second value
                const int h = threadIdx.x & 31;
                R.v1 = h < R.cnt ? omega * dinvA[col[p0 + b + h]] : (T)0;
            }
            pair_row_scaled<T, V>(R, min(kPairRow, n - b), L.half, tr, lane_off, acc);
        }
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const T zv = mul_rn(tv[q], dw);
            acc[q] = zv + dw * (tv[q] - acc[q]);
        }
        if (store) vstore<T, V>(zo + o, acc);
    }
}

// ------------------------------------------------------------------ row-per-lane tiles (sliced ELL)
// One workgroup per (tile, slice of M members).  The workgroup first copies the
// slice of every node value its rows read into LDS (all loads of a thread in
// flight before its LDS stores), then each wavefront takes one block of 64 rows,
// one row per lane: per entry the lane loads the entry's packed LDS offset and
// value(s) (coalesced: a block's entries are stored column-major; prefetched a
// chunk ahead) and the staged node with 16-byte LDS reads, and accumulates all
// M members of both components.  Entries are consumed in CSR order with the
// same operations as the other SpMM and Jacobi kernels, so results agree bitwise.
struct EllView {
    const int32_t *tile, *s2, *s1, *blk, *rows, *self;
    const int2* am;   // A entries: (LDS offset, value bits)
    const int4* bm;   // B^T / B entries: (LDS offset, first value bits, second value bits, 0)
};

constexpr int kEllChunk = 4;   // entries per prefetch chunk

struct EllMeta {
    int off[kEllChunk];
    float a[kEllChunk], b[kEllChunk];
};

// entries k0 ... k0 + kEllChunk - 1 (< K) of a lane whose entry k sits at e + 64 k
template <bool PAIR>
__device__ __forceinline__ void ell_meta(EllMeta& M, const EllView& E, int e, int k0, int K) {
#pragma unroll
    for (int i = 0; i < kEllChunk; ++i) {
        const int k = k0 + i;
        M.off[i] = 0;
        M.a[i] = 0.f;
        M.b[i] = 0.f;
        if (k < K) {
            if (PAIR) {
                const int4 q = E.bm[e + 64 * k];
                M.off[i] = q.x;
                M.a[i] = __int_as_float(q.y);
                M.b[i] = __int_as_float(q.z);
            } else {
                const int2 q = E.am[e + 64 * k];
                M.off[i] = q.x;
                M.a[i] = __int_as_float(q.y);
            }
        }
    }
}

// Copies the M-member slice (members j0 ...) of n2 velocity nodes (rows 2 node
// and 2 node + 1 of v2) to LDS slots of ell_p2_bytes(M) from offset 0, and of
// n1 pressure nodes (row node of v1) to slots of ell_p1_bytes(M) from offset
// dst1.  A P2 node is 2 M / 4 chunks of 16 bytes (component, 4 members), a P1
// node M / 4.  Branch-free so that all loads of a thread are in flight
// together: chunks past the end reload the first listed node and go to a
// 16-byte slot past the staged values.
template <int M, int NT>
__device__ __forceinline__ void ell_stage(unsigned char* lds, const int32_t* __restrict__ s2, int n2,
                                          const int32_t* __restrict__ s1, int n1, int dst1,
                                          const float* __restrict__ v2, const float* __restrict__ v1, int J, int j0) {
    constexpr int Q = M / 4;                 // chunks per component
    constexpr int LQ = Q == 4 ? 2 : 1;       // log2 Q
    constexpr int S2 = ell_p2_bytes(M), S1 = ell_p1_bytes(M);
    const int c2 = n2 * 2 * Q, tot = c2 + n1 * Q;
    const int spill = max(n2 * S2, dst1 + n1 * S1);
    for (int base = threadIdx.x; base < tot; base += 8 * NT) {
        int row[8], dst[8];
        bool one[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = base + k * NT;
            const bool is2 = i < c2, is1 = !is2 && i < tot;
            const int j = is2 ? i : (is1 ? i - c2 : 0);   // chunk within its kind
            const int sl = is1 ? (j >> LQ) : (j >> (LQ + 1));
            const int node = is1 ? s1[sl] : (n2 ? s2[sl] : s1[0]);
            one[k] = is1 || !n2;
            row[k] = one[k] ? node : 2 * node + ((j >> LQ) & 1);
            dst[k] = is2 ? sl * S2 + ((j >> LQ) & 1) * (M * 4) + (j & (Q - 1)) * 16
                         : (is1 ? dst1 + sl * S1 + (j & (Q - 1)) * 16 : spill);
        }
        float4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = base + k * NT;
            const int j = i < c2 ? i : (i < tot ? i - c2 : 0);
            const float* src = one[k] ? v1 : v2;
            v[k] = *(const float4*)(src + (int64_t)row[k] * J + j0 + (j & (Q - 1)) * 4);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) *(float4*)(lds + dst[k]) = v[k];
    }
}

// acc[c][m] += a * x[c][m] over entries of a lane (A entries: velocity node, both
// components); first holds the lane's first chunk, loaded by the caller
template <int M>
__device__ __forceinline__ void ell_rows_a(float (&acc)[2][M], const EllView& E, const unsigned char* lds, int e,
                                           int K, const EllMeta& first) {
    EllMeta cur = first, nxt;
    for (int k0 = 0; k0 < K; k0 += kEllChunk) {
        if (k0 + kEllChunk < K) ell_meta<false>(nxt, E, e, k0 + kEllChunk, K);
#pragma unroll
        for (int i = 0; i < kEllChunk; ++i) {
            if (k0 + i >= K) break;
            const float4* xs = (const float4*)(lds + cur.off[i]);
            const float a = cur.a[i];
#pragma unroll
            for (int q = 0; q < M / 2; ++q) {
                const float4 w = xs[q];
                float* r = &acc[q / (M / 4)][(q % (M / 4)) * 4];
                r[0] += a * w.x;
                r[1] += a * w.y;
                r[2] += a * w.z;
                r[3] += a * w.w;
            }
        }
        cur = nxt;
    }
}

template <int M>
__device__ __forceinline__ void ell_rows_a(float (&acc)[2][M], const EllView& E, const unsigned char* lds, int e,
                                           int K) {
    EllMeta first;
    ell_meta<false>(first, E, e, 0, K);
    ell_rows_a<M>(acc, E, lds, e, K, first);
}

// acc[0][m] += s a0 p[m], acc[1][m] += s a1 p[m] over B^T entries (pressure node), s = -1 if NEG
template <int M, bool NEG>
__device__ __forceinline__ void ell_rows_bt(float (&acc)[2][M], const EllView& E, const unsigned char* lds, int e,
                                            int K) {
    EllMeta cur, nxt;
    ell_meta<true>(cur, E, e, 0, K);
    for (int k0 = 0; k0 < K; k0 += kEllChunk) {
        if (k0 + kEllChunk < K) ell_meta<true>(nxt, E, e, k0 + kEllChunk, K);
#pragma unroll
        for (int i = 0; i < kEllChunk; ++i) {
            if (k0 + i >= K) break;
            const float4* ps = (const float4*)(lds + cur.off[i]);
            const float a0 = NEG ? -cur.a[i] : cur.a[i], a1 = NEG ? -cur.b[i] : cur.b[i];
#pragma unroll
            for (int q = 0; q < M / 4; ++q) {
                const float4 w = ps[q];
                acc[0][4 * q + 0] += a0 * w.x;
                acc[0][4 * q + 1] += a0 * w.y;
                acc[0][4 * q + 2] += a0 * w.z;
                acc[0][4 * q + 3] += a0 * w.w;
                acc[1][4 * q + 0] += a1 * w.x;
                acc[1][4 * q + 1] += a1 * w.y;
                acc[1][4 * q + 2] += a1 * w.z;
                acc[1][4 * q + 3] += a1 * w.w;
            }
        }
        cur = nxt;
    }
}

// y = S x, FP32, J a multiple of M; NW wavefronts per workgroup (>= blocks of any tile)
template <int M, int NW>
__global__ void __launch_bounds__(NW * 64) k_saddle_e(EllView E, const float* __restrict__ dp,
                                                      const float* __restrict__ x, float* __restrict__ y, int nP2,
                                                      int J, int MS) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int NT = NW * 64;
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int tile = (int)(bid / MS);
    const int j0 = (int)(bid % MS) * M;
    const int32_t* td = E.tile + 8 * tile;
    const int s2o = td[0], n2 = td[1], s1o = td[2], n1 = td[3], b0 = td[4], nb = td[5];
    // the first chunk of a lane's entries is requested before the staging, so
    // that its latency overlaps the staging's
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int32_t* bd = E.blk + 8 * (b0 + (wave < nb ? wave : 0));
    const int kind = bd[0], K1 = bd[2], K2 = bd[3], e1 = bd[4] + lane, e2 = bd[5] + lane, ro = bd[6];
    EllMeta first;
    if (wave < nb) {
        if (kind == 0)
            ell_meta<false>(first, E, e1, 0, K1);
        else
            ell_meta<true>(first, E, e1, 0, K1);
    }
    ell_stage<M, NT>(smem_raw, E.s2 + s2o, n2, E.s1 + s1o, n1, n2 * ell_p2_bytes(M), x,
                     x + 2 * (int64_t)nP2 * J, J, j0);
    __syncthreads();
    if (wave >= nb) return;
    const int row = E.rows[ro + lane];
    float acc[2][M];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[c][m] = 0.f;
    if (kind == 0) {
        ell_rows_a<M>(acc, E, smem_raw, e1, K1, first);
        ell_rows_bt<M, false>(acc, E, smem_raw, e2, K2);
        if (row >= 0) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float4* o = (float4*)(y + (2 * (int64_t)row + c) * J + j0);
#pragma unroll
                for (int q = 0; q < M / 4; ++q)
                    o[q] = make_float4(acc[c][4 * q], acc[c][4 * q + 1], acc[c][4 * q + 2], acc[c][4 * q + 3]);
            }
        }
    } else {
        // B rows: acc[0] = sum b_x x_0, acc[1] = sum b_y x_1 over the velocity nodes
        EllMeta cur = first, nxt;
        for (int k0 = 0; k0 < K1; k0 += kEllChunk) {
            if (k0 + kEllChunk < K1) ell_meta<true>(nxt, E, e1, k0 + kEllChunk, K1);
#pragma unroll
            for (int i = 0; i < kEllChunk; ++i) {
                if (k0 + i >= K1) break;
                const float4* xs = (const float4*)(smem_raw + cur.off[i]);
                const float a0 = cur.a[i], a1 = cur.b[i];
#pragma unroll
                for (int q = 0; q < M / 4; ++q) {
                    const float4 w = xs[q], u = xs[M / 4 + q];
                    acc[0][4 * q + 0] += a0 * w.x;
                    acc[0][4 * q + 1] += a0 * w.y;
                    acc[0][4 * q + 2] += a0 * w.z;
                    acc[0][4 * q + 3] += a0 * w.w;
                    acc[1][4 * q + 0] += a1 * u.x;
                    acc[1][4 * q + 1] += a1 * u.y;
                    acc[1][4 * q + 2] += a1 * u.z;
                    acc[1][4 * q + 3] += a1 * u.w;
                }
            }
            cur = nxt;
        }
        if (row >= 0) {
            const float d = dp[row];
            const float4* ps = (const float4*)(smem_raw + E.self[ro + lane]);
            float4* o = (float4*)(y + (2 * (int64_t)nP2 + row) * J + j0);
#pragma unroll
            for (int q = 0; q < M / 4; ++q) {
                const float4 w = ps[q];
                float r[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) r[t] = acc[0][4 * q + t] + acc[1][4 * q + t];
                r[0] += d * w.x;
                r[1] += d * w.y;
                r[2] += d * w.z;
                r[3] += d * w.w;
                o[q] = make_float4(r[0], r[1], r[2], r[3]);
            }
        }
    }
}

// Velocity-block Jacobi with row-per-lane tiles (operations as k_velo_h): FIRST
// stages the pressure slice of z_p and forms t = r_u - B^T z_p, z = w D^-1 t;
// the other sweeps stage the velocity slice of z and form z + w D^-1 (t - A z).
// Only the P2 row blocks (the first of a tile) are computed.
template <int M, bool FIRST, int NW>
__global__ void __launch_bounds__(NW * 64) k_velo_e(EllView E, const float* __restrict__ dinvA,
                                                    const float* __restrict__ in, const float* __restrict__ zp,
                                                    float* __restrict__ t, const float* __restrict__ z,
                                                    float* __restrict__ zo, int J, int MS, float omega) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int NT = NW * 64;
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int tile = (int)(bid / MS);
    const int j0 = (int)(bid % MS) * M;
    const int32_t* td = E.tile + 8 * tile;
    const int s2o = td[0], n2 = td[1], s1o = td[2], n1 = td[3], b0 = td[4], nb = td[5];
    if (FIRST)   // P1 slots from 0: entry offsets (past the P2 slots) are shifted back
        ell_stage<M, NT>(smem_raw, E.s2 + s2o, 0, E.s1 + s1o, n1, 0, zp, zp, J, j0);
    else
        ell_stage<M, NT>(smem_raw, E.s2 + s2o, n2, E.s1 + s1o, 0, 0, z, z, J, j0);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (wave >= nb) return;
    const int32_t* bd = E.blk + 8 * (b0 + wave);
    if (bd[0] != 0) return;
    const int K1 = bd[2], K2 = bd[3], e1 = bd[4] + lane, e2 = bd[5] + lane, ro = bd[6];
    const int row = E.rows[ro + lane];
    const unsigned char* lds = FIRST ? smem_raw - n2 * ell_p2_bytes(M) : smem_raw;
    float acc[2][M];
    const int64_t o = 2 * (int64_t)max(row, 0) * J + j0;
    if constexpr (FIRST) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float4* r = (const float4*)(in + o + (int64_t)c * J);
#pragma unroll
            for (int q = 0; q < M / 4; ++q) {
                const float4 w = row >= 0 ? r[q] : make_float4(0.f, 0.f, 0.f, 0.f);
                acc[c][4 * q] = w.x;
                acc[c][4 * q + 1] = w.y;
                acc[c][4 * q + 2] = w.z;
                acc[c][4 * q + 3] = w.w;
            }
        }
        ell_rows_bt<M, true>(acc, E, lds, e2, K2);
        if (row >= 0) {
            const float dw = omega * dinvA[row];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float4* ot = (float4*)(t + o + (int64_t)c * J);
                float4* oz = (float4*)(zo + o + (int64_t)c * J);
#pragma unroll
                for (int q = 0; q < M / 4; ++q) {
                    ot[q] = make_float4(acc[c][4 * q], acc[c][4 * q + 1], acc[c][4 * q + 2], acc[c][4 * q + 3]);
                    oz[q] = make_float4(acc[c][4 * q] * dw, acc[c][4 * q + 1] * dw, acc[c][4 * q + 2] * dw,
                                        acc[c][4 * q + 3] * dw);
                }
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m) acc[c][m] = 0.f;
        ell_rows_a<M>(acc, E, lds, e1, K1);
        if (row >= 0) {
            const float dw = omega * dinvA[row];
            const float4* zs = (const float4*)(lds + E.self[ro + lane]);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float4* tr = (const float4*)(t + o + (int64_t)c * J);
                float4* oz = (float4*)(zo + o + (int64_t)c * J);
#pragma unroll
                for (int q = 0; q < M / 4; ++q) {
                    const float4 tv = tr[q], zv = zs[(M / 4) * c + q];
                    float* a = &acc[c][4 * q];
                    oz[q] = make_float4(zv.x + dw * (tv.x - a[0]), zv.y + dw * (tv.y - a[1]),
                                        zv.z + dw * (tv.z - a[2]), zv.w + dw * (tv.w - a[3]));
                }
            }
        }
    }
}

// A values into the packed entries of a row-per-lane tiling: am[pos[p]].y = bits of src[p]
__global__ void __launch_bounds__(kBlock) k_ell_scatter(const float* __restrict__ src, const int32_t* __restrict__ pos,
                                                        int2* __restrict__ am, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) am[pos[p]].y = __float_as_int(src[p]);
}

// ------------------------------------------------------------------ multigrid kernels
// Packed-row CSR kernel for the pressure multigrid: LPR lanes per row, each
// lane V = 256 / (LPR sizeof(T)) consecutive members, so one load instruction
// fetches 64 / LPR member rows of a tile of MJ = 256 / sizeof(T) members.
// Lane h of a row's group first loads the row's h-th column and value; they
// are broadcast with ds_bpermute.  Longer rows than LPR entries go in chunks of LPR.
// MODE 0: y = A x ; 1: y += A x ; 2: y = b - A x ; 3: y = x + w dinv (b - A x) ;
// 4: y = w dinv b ; 5: the two first Jacobi sweeps from a zero guess,
// y = x1 + w dinv (b - A x1) with x1 = w dinv b formed on the fly (x unused);
// 6: the last sweep of MODE 3 written as the Schur part of the preconditioner,
// y = -(x + w dinv (b - A x)), and y = b on row pin (an identity row).
template <typename T, int MODE, int LPR>
__global__ void __launch_bounds__(kBlock) k_mg(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const T* __restrict__ val, const T* __restrict__ dinv,
                                               const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                               int n, int J, T omega, int pin) {
    constexpr int V = 256 / (LPR * (int)sizeof(T));
    constexpr int RPW = 64 / LPR;   // rows per wavefront
    const int lane = threadIdx.x & 63;
    const int slot = lane / LPR, h = lane % LPR;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int r = (int)((blk * (kBlock / 64) + (threadIdx.x >> 6)) * RPW + slot);
    const int j = blockIdx.y * (LPR * V) + h * V;
    const bool valid = r < n;
    int p0 = 0, cnt = 0;
    if (valid) {
        p0 = rp[r];
        cnt = rp[r + 1] - p0;
    }
    int nmax = 0;
#pragma unroll
    for (int g = 0; g < RPW; ++g) nmax = max(nmax, __builtin_amdgcn_readlane(cnt, g * LPR));
    T s[V];
#pragma unroll
    for (int q = 0; q < V; ++q) s[q] = 0;
    // longer rows than LPR entries go in chunks of LPR
    for (int base = 0; MODE != 4 && base < nmax; base += LPR) {
        int c = 0;
        T a = 0;
        if (base + h < cnt) {
            c = col[p0 + base + h];
            a = val[p0 + base + h];
        }
        const int lim = min(LPR, nmax - base);
        for (int t = 0; t < lim; t += 4) {
            T v[4][V];
            T w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int src = slot * LPR + min(t + i, LPR - 1);
                const int k = __builtin_amdgcn_ds_bpermute(src << 2, c);
                w[i] = half_bcast(a, src);
                if (base + t + i >= cnt) w[i] = 0;
                vload<T, V>(v[i], (MODE == 5 ? b : x) + (int64_t)k * J + j);
                if (MODE == 5) {
                    const T d = omega * dinv[k];
#pragma unroll
                    for (int q = 0; q < V; ++q) v[i][q] = d * v[i][q];
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int q = 0; q < V; ++q) s[q] += w[i] * v[i][q];
            }
        }
    }
    if (!valid) return;
    const int64_t o = (int64_t)r * J + j;
    T out[V];
    if (MODE == 0) {
#pragma unroll
        for (int q = 0; q < V; ++q) out[q] = s[q];
    } else if (MODE == 1) {
        vload<T, V>(out, y + o);
#pragma unroll
        for (int q = 0; q < V; ++q) out[q] += s[q];
    } else {
        T bv[V];
        vload<T, V>(bv, b + o);
        const T d = dinv ? dinv[r] : (T)0;
        if (MODE == 2) {
#pragma unroll
            for (int q = 0; q < V; ++q) out[q] = bv[q] - s[q];
        } else if (MODE == 3 || MODE == 6) {
            T xv[V];
            vload<T, V>(xv, x + o);
#pragma unroll
            for (int q = 0; q < V; ++q) out[q] = xv[q] + omega * d * (bv[q] - s[q]);
            if (MODE == 6) {
#pragma unroll
                for (int q = 0; q < V; ++q) out[q] = r == pin ? bv[q] : -out[q];
            }
        } else if (MODE == 4) {
#pragma unroll
            for (int q = 0; q < V; ++q) out[q] = omega * d * bv[q];
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) out[q] = omega * d * bv[q] + omega * d * (bv[q] - s[q]);
        }
    }
    vstore<T, V>(y + o, out);
}

// A fused step of a level's V-cycle as one sparse product on stacked inputs
// (the level's Dn or Up operator): y = A [x1; x2; x3], where columns below n1
// index x1, columns in [n1, n1 + n2) index x2 and the others x3.  Packed rows
// as in k_mg, 32 lanes per row, each lane 256 / (32 sizeof(T)) consecutive
// members; a row's entries go in chunks of 32 (one entry per lane, broadcast
// by ds_bpermute) with 8 member loads in flight.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mgf(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                const T* __restrict__ val, const T* __restrict__ x1,
                                                const T* __restrict__ x2, const T* __restrict__ x3, int n1, int n2,
                                                T* __restrict__ y, int n, int J) {
    constexpr int LPR = 32;
    constexpr int V = 256 / (LPR * (int)sizeof(T));
    constexpr int RPW = 64 / LPR;
    const int lane = threadIdx.x & 63;
    const int slot = lane / LPR, h = lane % LPR;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int r = (int)((blk * (kBlock / 64) + (threadIdx.x >> 6)) * RPW + slot);
    const int j = blockIdx.y * (LPR * V) + h * V;
    const bool valid = r < n;
    int p0 = 0, cnt = 0;
    if (valid) {
        p0 = rp[r];
        cnt = rp[r + 1] - p0;
    }
    int nmax = 0;
#pragma unroll
    for (int g = 0; g < RPW; ++g) nmax = max(nmax, __builtin_amdgcn_readlane(cnt, g * LPR));
    T s[V];
#pragma unroll
    for (int q = 0; q < V; ++q) s[q] = 0;
    for (int t0 = 0; t0 < nmax; t0 += LPR) {
        int c = 0;
        T a = 0;
        if (t0 + h < cnt) {
            c = col[p0 + t0 + h];
            a = val[p0 + t0 + h];
        }
        const int nt = min(LPR, nmax - t0);
        for (int t = 0; t < nt; t += 8) {
            T v[8][V];
            T w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int src = slot * LPR + min(t + i, LPR - 1);
                const int k = __builtin_amdgcn_ds_bpermute(src << 2, c);
                w[i] = half_bcast(a, src);
                if (t0 + t + i >= cnt) w[i] = 0;
                const T* xp = k < n1 ? x1 + (int64_t)k * J
                                     : (k < n1 + n2 ? x2 + (int64_t)(k - n1) * J : x3 + (int64_t)(k - n1 - n2) * J);
                vload<T, V>(v[i], xp + j);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
#pragma unroll
                for (int q = 0; q < V; ++q) s[q] += w[i] * v[i][q];
            }
        }
    }
    if (!valid) return;
    vstore<T, V>(y + (int64_t)r * J + j, s);
}

// Dense x = C b on the coarsest level (C: n x n row-major with row length ld, b and x: n x J),
// split over kDenseKS column ranges: a workgroup computes the partial product
// of a 64-row x 64-member block over one range (4 x 4 outputs per thread from
// 16-column slices staged in LDS); k_dense_sum adds the kDenseKS partials in a
// fixed order.
constexpr int kDenseKS = 16;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_part(const T* __restrict__ C, const T* __restrict__ b,
                                                       T* __restrict__ part, int n, int ld, int J) {
    __shared__ T As[16][64];   // [column][row]
    __shared__ T Bs[16][64];   // [column][member]
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int r0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int kc = (n + kDenseKS - 1) / kDenseKS;
    const int k0 = blockIdx.z * kc, k1 = min(n, k0 + kc);
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = 0;
    // the next 16-column slice is loaded into registers while the current one is used
    T ca[4], cb[4];
    auto fetch = [&](int kb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * kBlock;          // 0 .. 1023
            const int rr = idx >> 4, kk = idx & 15;
            const int r = r0 + rr, k = kb + kk;
            ca[e] = (r < n && k < k1) ? C[(int64_t)r * ld + k] : (T)0;
            const int bk = idx >> 6, bj = idx & 63;
            cb[e] = (kb + bk < k1 && j0 + bj < J) ? b[(int64_t)(kb + bk) * J + j0 + bj] : (T)0;
        }
    };
    if (k0 < k1) fetch(k0);
    for (int kb = k0; kb < k1; kb += 16) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * kBlock;
            As[idx & 15][idx >> 4] = ca[e];
            Bs[idx >> 6][idx & 63] = cb[e];
        }
        __syncthreads();
        if (kb + 16 < k1) fetch(kb + 16);
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            T av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                av[i] = As[kk][ty * 4 + i];
                bv[i] = Bs[kk][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] += av[i] * bv[q];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + ty * 4 + i;
        if (r >= n) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + tx * 4 + q;
            if (j < J) part[((int64_t)blockIdx.z * n + r) * J + j] = acc[i][q];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_sum(const T* __restrict__ part, T* __restrict__ x, int64_t nJ) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nJ) return;
    T s = part[i];
#pragma unroll
    for (int k = 1; k < kDenseKS; ++k) s += part[(int64_t)k * nJ + i];
    x[i] = s;
}

// The same product in FP32 on the matrix cores (J a multiple of 16, C zero-padded
// to ld x ld, ld a multiple of 16).  A workgroup of kDenseWaves wavefronts owns a
// 16-row x 16-member block of x; wavefront w takes an equal share of the
// 16-column blocks of C, loads kDenseBlocks of them (a row's 16 columns as four
// 16-byte loads across the lane groups, and the matching 16 rows of b) before
// its v_mfma_f32_16x16x4f32 steps, and the partial blocks are added in wavefront
// order through LDS.  Column k = 16 q + 4 g + s enters step s of block q in lane
// group g, for both operands.
constexpr int kDenseWaves = 16, kDenseBlocks = 5;
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kDenseWaves * 64) k_dense_mf(const float* __restrict__ C, const float* __restrict__ b,
                                                              float* __restrict__ x, int n, int ld, int J) {
    __shared__ float red[kDenseWaves][16][17];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const int nkb = ld / 16, per = (nkb + kDenseWaves - 1) / kDenseWaves;
    const int kb0 = min(nkb, w * per), kb1 = min(nkb, kb0 + per);
    const int g = lane >> 4, c = lane & 15;
    const float* arow = C + (int64_t)(r0 + c) * ld + 4 * g;
    floatx4_t d = {0.f, 0.f, 0.f, 0.f};
    for (int q0 = kb0; q0 < kb1; q0 += kDenseBlocks) {
        float4 a[kDenseBlocks];
        float bv[kDenseBlocks][4];
#pragma unroll
        for (int q = 0; q < kDenseBlocks; ++q) {
            const int kb = q0 + q < kb1 ? q0 + q : kb0;   // past the share: a reload left unused
            a[q] = *(const float4*)(arow + 16 * kb);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * kb + 4 * g + s;
                bv[q][s] = k < n ? b[(int64_t)k * J + j0 + c] : 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < kDenseBlocks; ++q) {
            if (q0 + q < kb1) {
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, bv[q][0], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].y, bv[q][1], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].z, bv[q][2], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].w, bv[q][3], d, 0, 0, 0);
            }
        }
    }
    // lane (g, c) holds rows 4 g ... 4 g + 3 of column c of the block
#pragma unroll
    for (int i = 0; i < 4; ++i) red[w][4 * g + i][c] = d[i];
    __syncthreads();
    if (threadIdx.x < 256) {
        const int row = threadIdx.x >> 4, col = threadIdx.x & 15;
        float sum = red[0][row][col];
        for (int q = 1; q < kDenseWaves; ++q) sum += red[q][row][col];
        if (r0 + row < n) x[(int64_t)(r0 + row) * J + j0 + col] = sum;
    }
}

// ------------------------------------------------------------------ LDS-staged node-row kernels
// One workgroup per (row tile, slice of JT = 32 VEC members).  The node values
// the tile's rows read are first copied into LDS with 16-byte loads
// ([node][component][JT] for velocities, [node][JT] for pressures).  Each
// wavefront then computes whole rows from LDS with lane = component * 32 +
// member group of VEC; a row's column offsets and values are uniform across
// the wavefront and come in through scalar loads.  Entries are consumed in CSR
// order, so the arithmetic matches the other kernels.
constexpr int kTileJ = 32;   // members of a slice per member per lane

struct TileView {
    const int32_t *r2_ptr, *r2, *r2_self, *r1_ptr, *r1, *r1_self, *s2_ptr, *s2, *s1_ptr, *s1;
    const int32_t *a_loc, *bt_loc, *b_loc;
};

// dst[(s * comps + c) * JT + q] = src[nodes[s] * node_stride + c * comp_stride + q], q < JT;
// 16-byte chunks, kStageU loads in flight per thread before the LDS stores
constexpr int kStageU = 4;
template <typename T, int JT>
__device__ __forceinline__ void stage_nodes(T* dst, const int32_t* __restrict__ nodes, int cnt,
                                            const T* __restrict__ src, int64_t node_stride, int comps,
                                            int64_t comp_stride, int nthreads) {
    constexpr int CH = 16 / (int)sizeof(T);
    constexpr int NCH = JT / CH;
    using V = typename VecT<T, CH>::type;
    const int total = cnt * comps * NCH;
    auto load = [&](int i) -> V {
        const int q = i % NCH;
        const int sc = i / NCH;
        const int c = sc % comps, s = sc / comps;
        return *(const V*)(src + (int64_t)nodes[s] * node_stride + c * comp_stride + q * CH);
    };
    int i = threadIdx.x;
    for (; i + (kStageU - 1) * nthreads < total; i += kStageU * nthreads) {
        V v[kStageU];
#pragma unroll
        for (int k = 0; k < kStageU; ++k) v[k] = load(i + k * nthreads);
#pragma unroll
        for (int k = 0; k < kStageU; ++k) *(V*)(dst + (int64_t)(i + k * nthreads) * CH) = v[k];
    }
    for (; i < total; i += nthreads) *(V*)(dst + (int64_t)i * CH) = load(i);
}

template <typename T, int VEC>
__device__ __forceinline__ void lds_load(T (&v)[VEC], const T* p) {
    if constexpr (VEC == 1) {
        v[0] = *p;
    } else {
        using V = typename VecT<T, VEC>::type;
        const V w = *(const V*)p;
        v[0] = w.x;
        v[1] = w.y;
    }
}

// acc[q] += sum over entries p in [p0, p1) of val[p] * base[loc[p] * stride + q]
template <typename T, int VEC>
__device__ __forceinline__ void lds_gather(const int32_t* __restrict__ loc, const T* __restrict__ val, int p0,
                                           int p1, const T* base, int stride, T (&acc)[VEC]) {
    int p = p0;
    for (; p + 4 <= p1; p += 4) {
        T v[4][VEC];
#pragma unroll
        for (int i = 0; i < 4; ++i) lds_load<T, VEC>(v[i], base + loc[p + i] * stride);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T a = val[p + i];
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] += a * v[i][q];
        }
    }
    for (; p < p1; ++p) {
        T v[VEC];
        lds_load<T, VEC>(v, base + loc[p] * stride);
        const T a = val[p];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] += a * v[q];
    }
}

// two values per entry (one per velocity component): acc0 with val[2p], acc1
// with val[2p + 1]; NEG subtracts
template <typename T, int VEC, bool NEG>
__device__ __forceinline__ void lds_gather2(const int32_t* __restrict__ loc, const T* __restrict__ val, int p0,
                                            int p1, const T* base, int stride, T (&acc0)[VEC], T (&acc1)[VEC]) {
    int p = p0;
    for (; p + 4 <= p1; p += 4) {
        T v[4][VEC];
#pragma unroll
        for (int i = 0; i < 4; ++i) lds_load<T, VEC>(v[i], base + loc[p + i] * stride);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T a0 = NEG ? -val[2 * (p + i)] : val[2 * (p + i)];
            const T a1 = NEG ? -val[2 * (p + i) + 1] : val[2 * (p + i) + 1];
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                acc0[q] += a0 * v[i][q];
                acc1[q] += a1 * v[i][q];
            }
        }
    }
    for (; p < p1; ++p) {
        T v[VEC];
        lds_load<T, VEC>(v, base + loc[p] * stride);
        const T a0 = NEG ? -val[2 * p] : val[2 * p];
        const T a1 = NEG ? -val[2 * p + 1] : val[2 * p + 1];
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            acc0[q] += a0 * v[q];
            acc1[q] += a1 * v[q];
        }
    }
}

struct TileLanes {
    int tile, j0, c, jj, wave;
};

template <int VEC>
__device__ __forceinline__ TileLanes tile_lanes(int MT) {
    TileLanes L;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    L.tile = (int)(blk / MT);
    L.j0 = (int)(blk % MT) * kTileJ * VEC;
    const int lane = threadIdx.x & 63;
    L.c = lane >> 5;
    L.jj = (lane & 31) * VEC;
    L.wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    return L;
}

// Row metadata of one wavefront's rows: lane i holds the i-th row the
// wavefront owns (rows base + wave + i NW of the tile), at most 64 rows.
struct WaveRows {
    int n;              // rows of this wavefront (uniform)
    int row, p0, p1, q0, q1;
};

__device__ __forceinline__ WaveRows wave_rows(const int32_t* __restrict__ rows, int rb, int re, int wave, int NW,
                                              const int32_t* __restrict__ rp0, const int32_t* __restrict__ rp1) {
    WaveRows W;
    const int lane = threadIdx.x & 63;
    W.n = re - rb > wave ? (re - rb - wave + NW - 1) / NW : 0;
    W.row = W.p0 = W.p1 = W.q0 = W.q1 = 0;
    if (lane < W.n) {
        W.row = rows[rb + wave + lane * NW];
        W.p0 = rp0[W.row];
        W.p1 = rp0[W.row + 1];
        if (rp1) {
            W.q0 = rp1[W.row];
            W.q1 = rp1[W.row + 1];
        }
    }
    return W;
}


// y = S x (MODE 0) or y = b - S x (MODE 1)
template <typename T, int VEC, int MODE, int NW>
__global__ void __launch_bounds__(NW * 64) k_saddle_lds(TileView tv, const int32_t* __restrict__ Arp,
                                                        const T* __restrict__ Aval, const int32_t* __restrict__ Btrp,
                                                        const T* __restrict__ Btval, const int32_t* __restrict__ Brp,
                                                        const T* __restrict__ Bval, const T* __restrict__ dp,
                                                        const T* __restrict__ x, const T* __restrict__ bvec,
                                                        T* __restrict__ y, int nP2, int J, int MT, int max_s2) {
    constexpr int JT = kTileJ * VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = (T*)smem_raw;
    T* ps = xs + (int64_t)max_s2 * 2 * JT;
    const TileLanes L = tile_lanes<VEC>(MT);
    const WaveRows W2 = wave_rows(tv.r2, tv.r2_ptr[L.tile], tv.r2_ptr[L.tile + 1], L.wave, NW, Arp, Btrp);
    const WaveRows W1 = wave_rows(tv.r1, tv.r1_ptr[L.tile], tv.r1_ptr[L.tile + 1], L.wave, NW, Brp, nullptr);
    const int s20 = tv.s2_ptr[L.tile], s10 = tv.s1_ptr[L.tile];
    const T* xp = x + 2 * (int64_t)nP2 * J;
    stage_nodes<T, JT>(xs, tv.s2 + s20, tv.s2_ptr[L.tile + 1] - s20, x + L.j0, 2 * (int64_t)J, 2, J, NW * 64);
    stage_nodes<T, JT>(ps, tv.s1 + s10, tv.s1_ptr[L.tile + 1] - s10, xp + L.j0, J, 1, 0, NW * 64);
    __syncthreads();
    const T* xsc = xs + L.c * JT + L.jj;
    const T* psc = ps + L.jj;
    for (int i = 0; i < W2.n; ++i) {
        T acc0[VEC], acc1[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc0[q] = 0;
        lds_gather<T, VEC>(tv.a_loc, Aval, rl(W2.p0, i), rl(W2.p1, i), xsc, 2 * JT, acc0);
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc1[q] = acc0[q];
        lds_gather2<T, VEC, false>(tv.bt_loc, Btval, rl(W2.q0, i), rl(W2.q1, i), psc, JT, acc0, acc1);
        const int64_t o = (2 * (int64_t)rl(W2.row, i) + L.c) * J + L.j0 + L.jj;
        T out[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) out[q] = L.c ? acc1[q] : acc0[q];
        if (MODE == 1) {
            T bv[VEC];
            vload<T, VEC>(bv, bvec + o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) out[q] = bv[q] - out[q];
        }
        vstore<T, VEC>(y + o, out);
    }
    const int r1b = tv.r1_ptr[L.tile] + L.wave;
    for (int i = 0; i < W1.n; ++i) {
        const int k = rl(W1.row, i);
        T acc0[VEC], acc1[VEC], out[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc0[q] = acc1[q] = 0;
        lds_gather2<T, VEC, false>(tv.b_loc, Bval, rl(W1.p0, i), rl(W1.p1, i), xsc, 2 * JT, acc0, acc1);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            out[q] = L.c ? acc1[q] : acc0[q];
            out[q] += __shfl_xor(out[q], 32, 64);   // the two velocity components' contributions
        }
        if (L.c == 0) {
            const T d = dp[k];
            T v[VEC];
            lds_load<T, VEC>(v, ps + tv.r1_self[r1b + i * NW] * JT + L.jj);
#pragma unroll
            for (int q = 0; q < VEC; ++q) out[q] += d * v[q];
            const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j0 + L.jj;
            if (MODE == 1) {
                T bv[VEC];
                vload<T, VEC>(bv, bvec + o);
#pragma unroll
                for (int q = 0; q < VEC; ++q) out[q] = bv[q] - out[q];
            }
            vstore<T, VEC>(y + o, out);
        }
    }
}

// velocity-block Jacobi (operations as k_velo_v).  FIRST stages the pressure
// part z_p, the other sweeps stage z.
template <typename T, int VEC, bool FIRST, int NW>
__global__ void __launch_bounds__(NW * 64) k_velo_lds(TileView tv, const int32_t* __restrict__ rp,
                                                      const T* __restrict__ val, const T* __restrict__ dinvA,
                                                      const T* __restrict__ in, const T* __restrict__ zp,
                                                      T* __restrict__ t, const T* __restrict__ z,
                                                      T* __restrict__ zo, int J, int MT, T omega) {
    constexpr int JT = kTileJ * VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = (T*)smem_raw;
    const TileLanes L = tile_lanes<VEC>(MT);
    const WaveRows W = wave_rows(tv.r2, tv.r2_ptr[L.tile], tv.r2_ptr[L.tile + 1], L.wave, NW, rp, nullptr);
    if (FIRST) {
        const int s10 = tv.s1_ptr[L.tile];
        stage_nodes<T, JT>(xs, tv.s1 + s10, tv.s1_ptr[L.tile + 1] - s10, zp + L.j0, J, 1, 0, NW * 64);
    } else {
        const int s20 = tv.s2_ptr[L.tile];
        stage_nodes<T, JT>(xs, tv.s2 + s20, tv.s2_ptr[L.tile + 1] - s20, z + L.j0, 2 * (int64_t)J, 2, J, NW * 64);
    }
    __syncthreads();
    const int rb = tv.r2_ptr[L.tile] + L.wave;
    for (int i = 0; i < W.n; ++i) {
        const int u = rl(W.row, i);
        const T dw = omega * dinvA[u];
        const int64_t o = (2 * (int64_t)u + L.c) * J + L.j0 + L.jj;
        T acc[VEC];
        if constexpr (FIRST) {
            T acc1[VEC];
            vload<T, VEC>(acc, in + o);   // r_u
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc1[q] = acc[q];
            lds_gather2<T, VEC, true>(tv.bt_loc, val, rl(W.p0, i), rl(W.p1, i), xs + L.jj, JT, acc, acc1);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = L.c ? acc1[q] : acc[q];
            vstore<T, VEC>(t + o, acc);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] *= dw;
            vstore<T, VEC>(zo + o, acc);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = 0;
            lds_gather<T, VEC>(tv.a_loc, val, rl(W.p0, i), rl(W.p1, i), xs + L.c * JT + L.jj, 2 * JT, acc);
            T tv_[VEC], zv[VEC];
            vload<T, VEC>(tv_, t + o);
            lds_load<T, VEC>(zv, xs + (tv.r2_self[rb + i * NW] * 2 + L.c) * JT + L.jj);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = zv[q] + dw * (tv_[q] - acc[q]);
            vstore<T, VEC>(zo + o, acc);
        }
    }
}

// ------------------------------------------------------------------ LDS-staged rows with staged entries
// As the LDS-staged kernels above, but the tile's CSR entries (local column
// index and value, gathered from the global value arrays in tile order) are
// staged into LDS beside the node values, so computing a row touches only LDS:
// the entry index is uniform across the wavefront (an LDS broadcast read), the
// node values are read per lane.  Entries are consumed in CSR order.
struct TileEnt {
    const int32_t *ta_rp, *ta_loc, *ta_gp, *tbt_rp, *tbt_loc, *tbt_gp, *tb_rp, *tb_loc, *tb_gp;
};
struct TileDims {
    int max_s2, max_s1, max_ea, max_ebt, max_eb;
};

// lane i < n holds the i-th row of this wavefront in tile order: its global row
// id and its entry bounds relative to the tile's first entry (e0)
struct WaveTRows {
    int n, row, p0, p1, q0, q1, self;
};

__device__ __forceinline__ WaveTRows wave_trows(int rb, int re, int wave, int NW, const int32_t* __restrict__ rows,
                                                const int32_t* __restrict__ rpa, int ea0,
                                                const int32_t* __restrict__ rpb, int eb0,
                                                const int32_t* __restrict__ selfs) {
    WaveTRows W;
    const int lane = threadIdx.x & 63;
    W.n = re - rb > wave ? (re - rb - wave + NW - 1) / NW : 0;
    W.row = W.p0 = W.p1 = W.q0 = W.q1 = W.self = 0;
    if (lane < W.n) {
        const int r = rb + wave + lane * NW;
        W.row = rows[r];
        W.p0 = rpa[r] - ea0;
        W.p1 = rpa[r + 1] - ea0;
        if (rpb) {
            W.q0 = rpb[r] - eb0;
            W.q1 = rpb[r + 1] - eb0;
        }
        if (selfs) W.self = selfs[r];
    }
    return W;
}

// copies cnt staged entries: loc[e] = tloc[e0 + e], val[NV e + v] = gval[NV gp[e0 + e] + v]
template <typename T, int NV>
__device__ __forceinline__ void stage_entries(int32_t* loc, T* val, const int32_t* __restrict__ tloc,
                                              const int32_t* __restrict__ tgp, const T* __restrict__ gval, int e0,
                                              int cnt, int nthreads) {
    for (int e = threadIdx.x; e < cnt; e += nthreads) {
        loc[e] = tloc[e0 + e];
        const int64_t g = tgp[e0 + e];   // -1: padding entry
#pragma unroll
        for (int v = 0; v < NV; ++v) val[NV * e + v] = g >= 0 ? gval[NV * g + v] : (T)0;
    }
}

// A whole row at once: its padded entries [e0, e0 + n4) (n4 a multiple of 4,
// at most 4 NG) are read 4 at a time (uniform LDS reads, broadcast to all
// lanes), then all node values, then the multiply-adds in entry order.
// acc0 += val . x; with PAIR also acc1 += val' . x (values val[2e], val[2e + 1]).
template <typename T, int VEC, int NG, bool PAIR, bool NEG>
__device__ __forceinline__ void lds_row_all(const int32_t* loc, const T* val, int e0, int n4, const T* base,
                                            int stride, T (&acc0)[VEC], T (&acc1)[VEC]) {
    int4 l[NG];
    T a0[NG][4], a1[NG][4];
    T v[NG][4][VEC];
#pragma unroll
    for (int g = 0; g < NG; ++g)
        if (4 * g < n4) {
            l[g] = *(const int4*)(loc + e0 + 4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (PAIR) {
                    a0[g][i] = val[2 * (e0 + 4 * g + i)];
                    a1[g][i] = val[2 * (e0 + 4 * g + i) + 1];
                } else {
                    a0[g][i] = val[e0 + 4 * g + i];
                }
            }
        }
#pragma unroll
    for (int g = 0; g < NG; ++g)
        if (4 * g < n4) {
            lds_load<T, VEC>(v[g][0], base + l[g].x * stride);
            lds_load<T, VEC>(v[g][1], base + l[g].y * stride);
            lds_load<T, VEC>(v[g][2], base + l[g].z * stride);
            lds_load<T, VEC>(v[g][3], base + l[g].w * stride);
        }
#pragma unroll
    for (int g = 0; g < NG; ++g)
        if (4 * g < n4) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T p0 = NEG ? -a0[g][i] : a0[g][i];
#pragma unroll
                for (int q = 0; q < VEC; ++q) acc0[q] += p0 * v[g][i][q];
                if (PAIR) {
                    const T p1 = NEG ? -a1[g][i] : a1[g][i];
#pragma unroll
                    for (int q = 0; q < VEC; ++q) acc1[q] += p1 * v[g][i][q];
                }
            }
        }
}

// y = S x (MODE 0) or y = b - S x (MODE 1)
template <typename T, int VEC, int MODE, int NW>
__global__ void __launch_bounds__(NW * 64) k_saddle_t(TileView tv, TileEnt te, TileDims d,
                                                      const T* __restrict__ Aval, const T* __restrict__ Btval,
                                                      const T* __restrict__ Bval, const T* __restrict__ dp,
                                                      const T* __restrict__ x, const T* __restrict__ bvec,
                                                      T* __restrict__ y, int nP2, int J, int MT) {
    constexpr int JT = kTileJ * VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = (T*)smem_raw;
    T* ps = xs + (int64_t)d.max_s2 * 2 * JT;
    T* av = ps + (int64_t)d.max_s1 * JT;
    T* btv = av + d.max_ea;
    T* bv = btv + 2 * d.max_ebt;
    int32_t* al = (int32_t*)(bv + 2 * d.max_eb);
    int32_t* btl = al + d.max_ea;
    int32_t* bl = btl + d.max_ebt;
    const TileLanes L = tile_lanes<VEC>(MT);
    const int r2b = tv.r2_ptr[L.tile], r2e = tv.r2_ptr[L.tile + 1];
    const int r1b = tv.r1_ptr[L.tile], r1e = tv.r1_ptr[L.tile + 1];
    const int ea0 = te.ta_rp[r2b], ebt0 = te.tbt_rp[r2b], eb0 = te.tb_rp[r1b];
    const WaveTRows W2 = wave_trows(r2b, r2e, L.wave, NW, tv.r2, te.ta_rp, ea0, te.tbt_rp, ebt0, nullptr);
    const WaveTRows W1 = wave_trows(r1b, r1e, L.wave, NW, tv.r1, te.tb_rp, eb0, nullptr, 0, tv.r1_self);
    const int s20 = tv.s2_ptr[L.tile], s10 = tv.s1_ptr[L.tile];
    const T* xp = x + 2 * (int64_t)nP2 * J;
    stage_nodes<T, JT>(xs, tv.s2 + s20, tv.s2_ptr[L.tile + 1] - s20, x + L.j0, 2 * (int64_t)J, 2, J, NW * 64);
    stage_nodes<T, JT>(ps, tv.s1 + s10, tv.s1_ptr[L.tile + 1] - s10, xp + L.j0, J, 1, 0, NW * 64);
    stage_entries<T, 1>(al, av, te.ta_loc, te.ta_gp, Aval, ea0, te.ta_rp[r2e] - ea0, NW * 64);
    stage_entries<T, 2>(btl, btv, te.tbt_loc, te.tbt_gp, Btval, ebt0, te.tbt_rp[r2e] - ebt0, NW * 64);
    stage_entries<T, 2>(bl, bv, te.tb_loc, te.tb_gp, Bval, eb0, te.tb_rp[r1e] - eb0, NW * 64);
    __syncthreads();
    const T* xsc = xs + L.c * JT + L.jj;
    const T* psc = ps + L.jj;
    for (int i = 0; i < W2.n; ++i) {
        T acc0[VEC], acc1[VEC], out[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc0[q] = 0;
        {
            const int a0 = rl(W2.p0, i);
            lds_row_all<T, VEC, kDeepA / 4, false, false>(al, av, a0, rl(W2.p1, i) - a0, xsc, 2 * JT, acc0, acc1);
        }
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc1[q] = acc0[q];
        {
            const int b0 = rl(W2.q0, i);
            lds_row_all<T, VEC, kDeepBt / 4, true, false>(btl, btv, b0, rl(W2.q1, i) - b0, psc, JT, acc0, acc1);
        }
        const int64_t o = (2 * (int64_t)rl(W2.row, i) + L.c) * J + L.j0 + L.jj;
#pragma unroll
        for (int q = 0; q < VEC; ++q) out[q] = L.c ? acc1[q] : acc0[q];
        if (MODE == 1) {
            T b_[VEC];
            vload<T, VEC>(b_, bvec + o);
#pragma unroll
            for (int q = 0; q < VEC; ++q) out[q] = b_[q] - out[q];
        }
        vstore<T, VEC>(y + o, out);
    }
    for (int i = 0; i < W1.n; ++i) {
        const int k = rl(W1.row, i);
        T acc0[VEC], acc1[VEC], out[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc0[q] = acc1[q] = 0;
        {
            const int q0 = rl(W1.p0, i);
            lds_row_all<T, VEC, kDeepA / 4, true, false>(bl, bv, q0, rl(W1.p1, i) - q0, xsc, 2 * JT, acc0, acc1);
        }
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            out[q] = L.c ? acc1[q] : acc0[q];
            out[q] += __shfl_xor(out[q], 32, 64);   // the two velocity components' contributions
        }
        if (L.c == 0) {
            const T dk = dp[k];
            T v[VEC];
            lds_load<T, VEC>(v, ps + rl(W1.self, i) * JT + L.jj);
#pragma unroll
            for (int q = 0; q < VEC; ++q) out[q] += dk * v[q];
            const int64_t o = (2 * (int64_t)nP2 + k) * J + L.j0 + L.jj;
            if (MODE == 1) {
                T b_[VEC];
                vload<T, VEC>(b_, bvec + o);
#pragma unroll
                for (int q = 0; q < VEC; ++q) out[q] = b_[q] - out[q];
            }
            vstore<T, VEC>(y + o, out);
        }
    }
}

// velocity-block Jacobi (operations as k_velo_v), rows and entries from LDS
template <typename T, int VEC, bool FIRST, int NW>
__global__ void __launch_bounds__(NW * 64) k_velo_t(TileView tv, TileEnt te, TileDims d, const T* __restrict__ val,
                                                    const T* __restrict__ dinvA, const T* __restrict__ in,
                                                    const T* __restrict__ zp, T* __restrict__ t,
                                                    const T* __restrict__ z, T* __restrict__ zo, int J, int MT,
                                                    T omega) {
    constexpr int JT = kTileJ * VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = (T*)smem_raw;
    const int nx = FIRST ? d.max_s1 * JT : d.max_s2 * 2 * JT;
    T* ev = xs + nx;
    int32_t* el = (int32_t*)(ev + (FIRST ? 2 * d.max_ebt : d.max_ea));
    const TileLanes L = tile_lanes<VEC>(MT);
    const int r2b = tv.r2_ptr[L.tile], r2e = tv.r2_ptr[L.tile + 1];
    const int32_t* rp = FIRST ? te.tbt_rp : te.ta_rp;
    const int e0 = rp[r2b];
    const WaveTRows W = wave_trows(r2b, r2e, L.wave, NW, tv.r2, rp, e0, nullptr, 0, FIRST ? nullptr : tv.r2_self);
    if (FIRST) {
        const int s10 = tv.s1_ptr[L.tile];
        stage_nodes<T, JT>(xs, tv.s1 + s10, tv.s1_ptr[L.tile + 1] - s10, zp + L.j0, J, 1, 0, NW * 64);
        stage_entries<T, 2>(el, ev, te.tbt_loc, te.tbt_gp, val, e0, rp[r2e] - e0, NW * 64);
    } else {
        const int s20 = tv.s2_ptr[L.tile];
        stage_nodes<T, JT>(xs, tv.s2 + s20, tv.s2_ptr[L.tile + 1] - s20, z + L.j0, 2 * (int64_t)J, 2, J, NW * 64);
        stage_entries<T, 1>(el, ev, te.ta_loc, te.ta_gp, val, e0, rp[r2e] - e0, NW * 64);
    }
    __syncthreads();
    for (int i = 0; i < W.n; ++i) {
        const int u = rl(W.row, i);
        const T dw = omega * dinvA[u];
        const int64_t o = (2 * (int64_t)u + L.c) * J + L.j0 + L.jj;
        T acc[VEC];
        if constexpr (FIRST) {
            T acc1[VEC];
            vload<T, VEC>(acc, in + o);   // r_u
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc1[q] = acc[q];
            const int e0_ = rl(W.p0, i);
            lds_row_all<T, VEC, kDeepBt / 4, true, true>(el, ev, e0_, rl(W.p1, i) - e0_, xs + L.jj, JT, acc, acc1);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = L.c ? acc1[q] : acc[q];
            vstore<T, VEC>(t + o, acc);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] *= dw;
            vstore<T, VEC>(zo + o, acc);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = 0;
            T unused[VEC];
            const int e0_ = rl(W.p0, i);
            lds_row_all<T, VEC, kDeepA / 4, false, false>(el, ev, e0_, rl(W.p1, i) - e0_, xs + L.c * JT + L.jj, 2 * JT,
                                                          acc, unused);
            T tv_[VEC], zv[VEC];
            vload<T, VEC>(tv_, t + o);
            lds_load<T, VEC>(zv, xs + (rl(W.self, i) * 2 + L.c) * JT + L.jj);
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[q] = zv[q] + dw * (tv_[q] - acc[q]);
            vstore<T, VEC>(zo + o, acc);
        }
    }
}

// ------------------------------------------------------------------ velocity block Jacobi
// first sweep: t = r_u - B^T z_p ; z = w D^{-1} t
template <typename T>
__global__ void __launch_bounds__(kBlock) k_velo_first(const int32_t* __restrict__ Btrp, const int32_t* __restrict__ Btcol,
                                                       const T* __restrict__ Btval, const T* __restrict__ dinvA,
                                                       const T* __restrict__ r, const T* __restrict__ zp,
                                                       T* __restrict__ t, T* __restrict__ z, int nP2, int J, int JP,
                                                       T omega) {
    Lanes L = lanes(JP);
    const int64_t i = L.unit;
    if (i >= nP2) return;
    const int32_t b0 = Btrp[i], b1 = Btrp[i + 1];
    const T dw = omega * dinvA[i];
    for (int j = L.j0; j < J; j += JP) {
        T s0 = r[(2 * i) * J + j], s1 = r[(2 * i + 1) * J + j];
        for (int32_t p = b0; p < b1; ++p) {
            const T pv = zp[(int64_t)Btcol[p] * J + j];
            s0 -= Btval[2 * p] * pv;
            s1 -= Btval[2 * p + 1] * pv;
        }
        t[(2 * i) * J + j] = s0;
        t[(2 * i + 1) * J + j] = s1;
        z[(2 * i) * J + j] = dw * s0;
        z[(2 * i + 1) * J + j] = dw * s1;
    }
}

// later sweeps: zo = z + w D^{-1} (t - A z)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_velo_sweep(const int32_t* __restrict__ Arp, const int32_t* __restrict__ Acol,
                                                       const T* __restrict__ Aval, const T* __restrict__ dinvA,
                                                       const T* __restrict__ t, const T* __restrict__ z,
                                                       T* __restrict__ zo, int nP2, int J, int JP, T omega) {
    Lanes L = lanes(JP);
    const int64_t i = L.unit;
    if (i >= nP2) return;
    const int32_t a0 = Arp[i], a1 = Arp[i + 1];
    const T dw = omega * dinvA[i];
    for (int j = L.j0; j < J; j += JP) {
        T s0 = 0, s1 = 0;
        for (int32_t p = a0; p < a1; ++p) {
            const int64_t k = Acol[p];
            const T a = Aval[p];
            s0 += a * z[(2 * k) * J + j];
            s1 += a * z[(2 * k + 1) * J + j];
        }
        const T z0 = z[(2 * i) * J + j], z1 = z[(2 * i + 1) * J + j];
        zo[(2 * i) * J + j] = z0 + dw * (t[(2 * i) * J + j] - s0);
        zo[(2 * i + 1) * J + j] = z1 + dw * (t[(2 * i + 1) * J + j] - s1);
    }
}

// ------------------------------------------------------------------ scalar CSR (multigrid)
// MODE 0: y = A x ; MODE 1: y += A x ; MODE 2: y = b - A x ;
// MODE 3: y = x + w dinv (b - A x) ; MODE 4: y = w dinv b (x unused) ;
// MODE 5: MODE 4 followed by MODE 3 in one pass (x unused)
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_csr(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                const T* __restrict__ val, const T* __restrict__ dinv,
                                                const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                                int64_t n, int J, int JP, T omega) {
    Lanes L = lanes(JP);
    const int64_t r = L.unit;
    if (r >= n) return;
    const int32_t p0 = rp[r], p1 = rp[r + 1];
    for (int j = L.j0; j < J; j += JP) {
        T s = 0;
        if (MODE == 5)
            for (int32_t p = p0; p < p1; ++p) {
                const int64_t k = col[p];
                s += val[p] * (omega * dinv[k] * b[k * J + j]);
            }
        else if (MODE != 4)
            for (int32_t p = p0; p < p1; ++p) s += val[p] * x[(int64_t)col[p] * J + j];
        const int64_t o = r * J + j;
        if (MODE == 0) y[o] = s;
        if (MODE == 1) y[o] += s;
        if (MODE == 2) y[o] = b[o] - s;
        if (MODE == 3) y[o] = x[o] + omega * dinv[r] * (b[o] - s);
        if (MODE == 4) y[o] = omega * dinv[r] * b[o];
        if (MODE == 5) y[o] = omega * dinv[r] * b[o] + omega * dinv[r] * (b[o] - s);
    }
}

// Schur part from two V-cycles: z_p = -(x1 + x2), the pinned row keeping r_p
template <typename T>
__global__ void __launch_bounds__(kBlock) k_schur2(const T* __restrict__ x1, const T* __restrict__ x2,
                                                   const T* __restrict__ rp, int pin, T* __restrict__ zp, int64_t nP1,
                                                   int J) {
    for (int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x; o < nP1 * J; o += (int64_t)gridDim.x * kBlock)
        zp[o] = (o / J == pin) ? rp[o] : -(x1[o] + x2[o]);
}

// z_p = -x_mg (x_mg ~ S_hat^{-1} r_p from the V-cycle); the pinned row is an
// identity row of S, so there z_p = r_p
template <typename T>
__global__ void __launch_bounds__(kBlock) k_schur(const T* __restrict__ xmg, const T* __restrict__ rp, int pin,
                                                  T* __restrict__ zp, int nP1, int J, int JP) {
    Lanes L = lanes(JP);
    const int64_t k = L.unit;
    if (k >= nP1) return;
    for (int j = L.j0; j < J; j += JP) {
        const int64_t o = k * J + j;
        zp[o] = (k == pin) ? rp[o] : -xmg[o];
    }
}

// ------------------------------------------------------------------ column reductions
// Column (= member) reductions over the rows of (n x J) blocks.  Mapping: each
// thread owns VEC consecutive members of one row (vector loads); CW threads
// cover a row's members, RG = 256 / CW rows are processed side by side and the
// grid strides over the rows.  Per-block partials are stored member-major,
// partial[q * nblk + block], and summed by k_reduce in a fixed order, so the
// results do not depend on scheduling.
template <typename T, int VEC>
struct VecT;
template <>
struct VecT<float, 4> {
    using type = float4;
};
template <>
struct VecT<float, 2> {
    using type = float2;
};
template <>
struct VecT<float, 1> {
    using type = float;
};
template <>
struct VecT<double, 2> {
    using type = double2;
};
template <>
struct VecT<double, 1> {
    using type = double;
};

template <typename T, int VEC>
__device__ __forceinline__ void vload(T (&v)[VEC], const T* p) {
    using V = typename VecT<T, VEC>::type;
    *reinterpret_cast<V*>(v) = *reinterpret_cast<const V*>(p);
}
template <typename T, int VEC>
__device__ __forceinline__ void vstore(T* p, const T (&v)[VEC]) {
    using V = typename VecT<T, VEC>::type;
    *reinterpret_cast<V*>(p) = *reinterpret_cast<const V*>(v);
}

// Compiler-only ordering point (emits no code) for a software-pipelined row
// loop: the registers of the row about to be used are marked as produced here,
// so the work on them cannot move above the next row's loads issued before this
// point, and those loads cannot move below it (memory clobber).
template <typename T, int VEC>
__device__ __forceinline__ void settle(T (&v)[VEC]) {
#pragma unroll
    for (int u = 0; u < VEC; ++u) asm volatile("" : "+v"(v[u])::"memory");
}

// vload through a global-address-space pointer: for block pointers read from a
// pointer array, which the compiler would otherwise load as flat accesses
template <typename T, int VEC>
__device__ __forceinline__ void gload(T (&v)[VEC], const T* p) {
    using GV = T __attribute__((ext_vector_type(VEC)));
    using GP = const GV __attribute__((address_space(1)))*;
    const GV x = *(GP)(p);
#pragma unroll
    for (int u = 0; u < VEC; ++u) v[u] = x[u];
}

struct ColMap {
    int tx, ty, RG, jb;
    bool ok;
};

__device__ __forceinline__ ColMap colmap(int CW, int VEC, int J) {
    ColMap c;
    c.tx = threadIdx.x % CW;
    c.ty = threadIdx.x / CW;
    c.RG = kBlock / CW;
    c.jb = (blockIdx.y * CW + c.tx) * VEC;
    c.ok = (c.ty < c.RG) && (c.jb < J);
    return c;
}

// block-level sum over the RG row groups of one value per thread; thread ty == 0
// returns the column sum
__device__ __forceinline__ double block_colsum(double v, const ColMap& c, double* red, int CW) {
    red[threadIdx.x] = v;
    __syncthreads();
    double s = 0.0;
    if (c.ty == 0)
        for (int g = 0; g < c.RG; ++g) s += red[g * CW + c.tx];
    __syncthreads();
    return s;
}

// Column sums of NV values per thread at once: value q of thread (tx, ty) is
// summed over the RG row groups in row-group order (as block_colsum) and
// out(q, tx, sum) is called once for every q and every tx < CW whose columns
// exist. Up to kColsumBatch values share one pass through LDS (red holds
// kColsumBatch * kBlock doubles), and the sums of a pass are spread over the
// whole block instead of the threads of row group 0.
constexpr int kColsumBatch = 8;

template <int NV, int VEC, typename Out>
__device__ __forceinline__ void block_colsums(const double (&v)[NV], const ColMap& c, double* red, int CW, int J,
                                              Out out) {
    constexpr int K = NV < kColsumBatch ? NV : kColsumBatch;
#pragma unroll
    for (int q0 = 0; q0 < NV; q0 += K) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (q0 + k < NV) red[k * kBlock + threadIdx.x] = v[q0 + k];
        __syncthreads();
        for (int o = threadIdx.x; o < K * CW; o += kBlock) {
            const int k = o / CW, tx = o - k * CW;
            if (q0 + k < NV && ((int)blockIdx.y * CW + tx) * VEC < J) {
                double sum = 0.0;
                for (int g = 0; g < c.RG; ++g) sum += red[k * kBlock + g * CW + tx];
                out(q0 + k, tx, sum);
            }
        }
        __syncthreads();
    }
}

// partial[((c0 + i) * J + j) * nblk + block] = sum over rows of V_i[r, j] * w[r, j], i < NB;
// with WW also sum over rows of w[r, j]^2 at i = NB.  NB is the exact count, so
// all loads of an iteration are issued before the products.
template <typename T, int VEC, int NB, bool WW = false>
__global__ void __launch_bounds__(kBlock) k_dots(const T* const* __restrict__ V, int c0, const T* __restrict__ w,
                                                 int64_t n, int J, int CW, double* __restrict__ partial) {
    __shared__ double red[kColsumBatch * kBlock];
    constexpr int NA = (NB + (WW ? 1 : 0)) * VEC;
    const ColMap c = colmap(CW, VEC, J);
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    if (c.ok && n > 0) {
        const T* vp[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) vp[i] = V[c0 + i];
        // Two register sets in turn: the next row's loads are issued before the
        // current row's products. The trip count is the block's (uniform), rows
        // past the end are re-reads of row n - 1 that add nothing.
        const int64_t stride = (int64_t)gridDim.x * c.RG;
        const int64_t r0 = (int64_t)blockIdx.x * c.RG;
        const int64_t trips = r0 < n ? (n - r0 + stride - 1) / stride : 0;
        int64_t r = r0 + c.ty;
        T wa[VEC], va[NB][VEC], wb[VEC], vb[NB][VEC];
        auto load = [&](int64_t rr, T (&w_)[VEC], T (&v_)[NB][VEC]) {
            const int64_t o = (rr < n ? rr : n - 1) * J + c.jb;
            gload<T, VEC>(w_, w + o);
#pragma unroll
            for (int i = 0; i < NB; ++i) gload<T, VEC>(v_[i], vp[i] + o);
        };
        auto hold = [&](T (&w_)[VEC], T (&v_)[NB][VEC]) {
            settle<T, VEC>(w_);
#pragma unroll
            for (int i = 0; i < NB; ++i) settle<T, VEC>(v_[i]);
        };
        auto add = [&](int64_t rr, const T (&w_)[VEC], const T (&v_)[NB][VEC]) {
            const bool live = rr < n;
            T wz[VEC];
#pragma unroll
            for (int u = 0; u < VEC; ++u) wz[u] = live ? w_[u] : T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int u = 0; u < VEC; ++u) acc[i * VEC + u] += (double)v_[i][u] * (double)wz[u];
            if (WW) {
#pragma unroll
                for (int u = 0; u < VEC; ++u) acc[NB * VEC + u] += (double)wz[u] * (double)wz[u];
            }
        };
        if (trips > 0) load(r, wa, va);
        for (int64_t k = 0; k < trips; k += 2) {
            load(r + stride, wb, vb);
            hold(wa, va);
            add(r, wa, va);
            r += stride;
            load(r + stride, wa, va);
            hold(wb, vb);
            add(r, wb, vb);
            r += stride;
        }
    }
    const int64_t nblk = gridDim.x;
    block_colsums<NA, VEC>(acc, c, red, CW, J,
                                 [&](int q, int tx, double sum) {
                                     const int i = q / VEC, u = q - i * VEC;
                                     const int64_t j = ((int64_t)blockIdx.y * CW + tx) * VEC + u;
                                     partial[((int64_t)(c0 + i) * J + j) * nblk + blockIdx.x] = sum;
                                 });
}

// w -= sum_{i<NB} h[(c0 + i) J + j] V_{c0 + i}; with LAST also partial[j * nblk +
// block] = sum over rows of w^2 (store = 0: the norm only, w left as it was);
// with scale the result is stored divided by scale[j] (0 where scale[j] is 0).  NB is the exact count (all loads of an
// iteration issued before the arithmetic); longer updates run in chunks, which
// perform the same operations in the same order.
template <typename T, int VEC, int NB, bool LAST>
__global__ void __launch_bounds__(kBlock) k_update(const T* const* __restrict__ V, int c0, const double* __restrict__ h,
                                                   T* __restrict__ w, int64_t n, int J, int CW,
                                                   double* __restrict__ partial, int store = 1,
                                                   const double* __restrict__ scale = nullptr) {
    __shared__ double red[kColsumBatch * kBlock];
    const ColMap c = colmap(CW, VEC, J);
    double acc[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
    if (c.ok) {
        T hh[NB][VEC];
        const T* vp[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            vp[i] = V[c0 + i];
#pragma unroll
            for (int u = 0; u < VEC; ++u) hh[i][u] = (T)h[(int64_t)(c0 + i) * J + c.jb + u];
        }
        double f[VEC];
#pragma unroll
        for (int u = 0; u < VEC; ++u) f[u] = scale ? scale[c.jb + u] : 1.0;
        // Two register sets in turn: the next row's loads are issued before the
        // current row is updated. The trip count is the block's (uniform), rows
        // past the end are re-reads of row n - 1 that store and add nothing.
        const int64_t stride = (int64_t)gridDim.x * c.RG;
        const int64_t r0 = (int64_t)blockIdx.x * c.RG;
        const int64_t trips = r0 < n ? (n - r0 + stride - 1) / stride : 0;
        int64_t r = r0 + c.ty;
        T wa[VEC], va[NB][VEC], wb[VEC], vb[NB][VEC];
        auto load = [&](int64_t rr, T (&w_)[VEC], T (&v_)[NB][VEC]) {
            const int64_t o = (rr < n ? rr : n - 1) * J + c.jb;
            gload<T, VEC>(w_, w + o);
#pragma unroll
            for (int i = 0; i < NB; ++i) gload<T, VEC>(v_[i], vp[i] + o);
        };
        auto hold = [&](T (&w_)[VEC], T (&v_)[NB][VEC]) {
            settle<T, VEC>(w_);
#pragma unroll
            for (int i = 0; i < NB; ++i) settle<T, VEC>(v_[i]);
        };
        auto update = [&](int64_t rr, T (&w_)[VEC], const T (&v_)[NB][VEC]) {
            const bool live = rr < n;
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int u = 0; u < VEC; ++u) w_[u] -= hh[i][u] * v_[i][u];
            if (live && store) {
                if (scale) {   // as k_scale_cols_v with invert
                    T o[VEC];
#pragma unroll
                    for (int u = 0; u < VEC; ++u) o[u] = (T)(f[u] > 0.0 ? (double)w_[u] / f[u] : 0.0);
                    vstore<T, VEC>(w + rr * J + c.jb, o);
                } else {
                    vstore<T, VEC>(w + rr * J + c.jb, w_);
                }
            }
            if (LAST) {
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    const T wl = live ? w_[u] : T(0);
                    acc[u] += (double)wl * (double)wl;
                }
            }
        };
        if (trips > 0) load(r, wa, va);
        for (int64_t k = 0; k < trips; k += 2) {
            load(r + stride, wb, vb);
            hold(wa, va);
            update(r, wa, va);
            r += stride;
            load(r + stride, wa, va);
            hold(wb, vb);
            update(r, wb, vb);
            r += stride;
        }
    }
    if (LAST) {
        const int64_t nblk = gridDim.x;
        block_colsums<VEC, VEC>(acc, c, red, CW, J, [&](int u, int tx, double sum) {
            partial[(((int64_t)blockIdx.y * CW + tx) * VEC + u) * nblk + blockIdx.x] = sum;
        });
    }
}

// partial[j * nblk + block] = sum over rows of a[r, j]^2 (FP64 blocks)
template <int VEC>
__global__ void __launch_bounds__(kBlock) k_colsq(const double* __restrict__ a, int64_t n, int J, int CW,
                                                  double* __restrict__ partial) {
    __shared__ double red[kColsumBatch * kBlock];
    const ColMap c = colmap(CW, VEC, J);
    double acc[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
    if (c.ok)
        for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG) {
            double v[VEC];
            vload<double, VEC>(v, a + r * J + c.jb);
#pragma unroll
            for (int u = 0; u < VEC; ++u) acc[u] += v[u] * v[u];
        }
    const int64_t nblk = gridDim.x;
    block_colsums<VEC, VEC>(acc, c, red, CW, J, [&](int u, int tx, double sum) {
        partial[(((int64_t)blockIdx.y * CW + tx) * VEC + u) * nblk + blockIdx.x] = sum;
    });
}

// u = sum_{i<NB} y[(c0 + i) J + j] V_{c0 + i}, added to u unless FIRST (chunks of an
// NB-exact combination, as k_update); with x64 the result is added to the FP64
// x instead of being stored (the last chunk of x += Z y)
template <typename T, int VEC, int NB, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_combine(const T* const* __restrict__ V, int c0, const double* __restrict__ yv,
                                                    T* __restrict__ u, int64_t n, int J, int CW,
                                                    double* __restrict__ x64 = nullptr) {
    const ColMap c = colmap(CW, VEC, J);
    if (!c.ok) return;
    T yy[NB][VEC];
    const T* vp[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        vp[i] = V[c0 + i];
#pragma unroll
        for (int q = 0; q < VEC; ++q) yy[i][q] = (T)yv[(int64_t)(c0 + i) * J + c.jb + q];
    }
    // Two register sets in turn: the next row's loads are issued before the
    // current row is combined. The trip count is the block's (uniform), rows past
    // the end are re-reads of row n - 1 that store nothing.
    const int64_t stride = (int64_t)gridDim.x * c.RG;
    const int64_t r0 = (int64_t)blockIdx.x * c.RG;
    const int64_t trips = r0 < n ? (n - r0 + stride - 1) / stride : 0;
    int64_t r = r0 + c.ty;
    T sa[VEC], va[NB][VEC], sb[VEC], vb[NB][VEC];
    auto load = [&](int64_t rr, T (&s_)[VEC], T (&v_)[NB][VEC]) {
        const int64_t o = (rr < n ? rr : n - 1) * J + c.jb;
        if (FIRST) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) s_[q] = 0;
        } else {
            gload<T, VEC>(s_, u + o);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) gload<T, VEC>(v_[i], vp[i] + o);
    };
    auto hold = [&](T (&s_)[VEC], T (&v_)[NB][VEC]) {
        settle<T, VEC>(s_);
#pragma unroll
        for (int i = 0; i < NB; ++i) settle<T, VEC>(v_[i]);
    };
    auto combine = [&](int64_t rr, T (&s_)[VEC], const T (&v_)[NB][VEC]) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < VEC; ++q) s_[q] += yy[i][q] * v_[i][q];
        if (rr >= n) return;
        if (!x64) {
            vstore<T, VEC>(u + rr * J + c.jb, s_);
        } else if constexpr (VEC % 2 == 0) {   // x += u in FP64 instead of storing u (as k_add_to64)
#pragma unroll
            for (int q = 0; q < VEC; q += 2) {
                double2* xp = (double2*)(x64 + rr * J + c.jb + q);
                double2 xv = *xp;
                xv.x += (double)s_[q];
                xv.y += (double)s_[q + 1];
                *xp = xv;
            }
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) x64[rr * J + c.jb + q] += (double)s_[q];
        }
    };
    if (trips > 0) load(r, sa, va);
    for (int64_t k = 0; k < trips; k += 2) {
        load(r + stride, sb, vb);
        hold(sa, va);
        combine(r, sa, va);
        r += stride;
        load(r + stride, sa, va);
        hold(sb, vb);
        combine(r, sb, vb);
        r += stride;
    }
}

// out[q] = sum_b partial[q * nblk + b], one wavefront per output, fixed order
// (strided lane sums, then a butterfly); optional square root
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partial, int nblk, int64_t width,
                                                   double* __restrict__ out, int take_sqrt) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    double s = 0.0;
    if (q < width)
        for (int b = lane; b < nblk; b += 64) s += partial[q * nblk + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (q < width && lane == 0) out[q] = take_sqrt ? sqrt(s) : s;
}

// elementwise helpers
template <typename TI, typename TO>
__global__ void __launch_bounds__(kBlock) k_scale_cols(const TI* __restrict__ a, const double* __restrict__ s, int invert,
                                                       TO* __restrict__ out, int64_t n, int J) {
    int64_t idx = ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    int64_t tot = n * J;
    for (; idx < tot; idx += (int64_t)gridDim.x * kBlock) {
        int j = (int)(idx % J);
        double f = s[j];
        double v = (double)a[idx];
        double r;
        if (invert)
            r = (f > 0.0) ? v / f : 0.0;
        else
            r = v * f;
        out[idx] = (TO)r;
    }
}

// as k_scale_cols with VEC consecutive members per thread (J a multiple of VEC):
// out[r, j] = a[r, j] / s[j] (invert; 0 where s[j] <= 0) or a[r, j] s[j]
template <typename TI, typename TO, int VEC>
__global__ void __launch_bounds__(kBlock) k_scale_cols_v(const TI* __restrict__ a, const double* __restrict__ s,
                                                         int invert, TO* __restrict__ out, int64_t n, int J, int CW) {
    const ColMap c = colmap(CW, VEC, J);
    if (!c.ok) return;
    double f[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) f[u] = s[c.jb + u];
    for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG) {
        TI v[VEC];
        TO o[VEC];
        vload<TI, VEC>(v, a + r * J + c.jb);
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
            const double x = (double)v[u];
            o[u] = (TO)(invert ? (f[u] > 0.0 ? x / f[u] : 0.0) : x * f[u]);
        }
        vstore<TO, VEC>(out + r * J + c.jb, o);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_add_to64(double* __restrict__ x, const T* __restrict__ d, int64_t tot) {
    int64_t idx = ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    for (; idx < tot; idx += (int64_t)gridDim.x * kBlock) x[idx] += (double)d[idx];
}

// per member: g = [beta, 0, ...]
__global__ void k_init_g(double* __restrict__ g, const double* __restrict__ beta, int m1, int J) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    for (int i = 0; i < m1; ++i) g[i * J + j] = 0.0;
    g[j] = beta[j];
}

// Givens step k for member j (FP64): rotate column k of H (hv[i * hs], i <= k,
// with hnj the new subdiagonal entry), new rotation, update g and the residual
// estimate
__device__ __forceinline__ void givens_step(double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                                            double* __restrict__ g, const double* hv, int hs, double hnj,
                                            double* __restrict__ res, int k, int m, int J, int j) {
    double h[kMaxRestart + 1];
    for (int i = 0; i <= k; ++i) h[i] = hv[i * hs];
    h[k + 1] = hnj;
    for (int i = 0; i < k; ++i) {
        double c = cs[i * J + j], s = sn[i * J + j];
        double t = c * h[i] + s * h[i + 1];
        h[i + 1] = -s * h[i] + c * h[i + 1];
        h[i] = t;
    }
    double a = h[k], b = h[k + 1];
    double c, s;
    if (a == 0.0 && b == 0.0) {
        c = 1.0;
        s = 0.0;
        h[k] = 1.0;     // inactive column: keeps the triangular solve defined (g_k is 0 here)
    } else {
        double r = hypot(a, b);
        c = a / r;
        s = b / r;
        h[k] = r;
    }
    cs[k * J + j] = c;
    sn[k * J + j] = s;
    for (int i = 0; i <= k; ++i) H[((int64_t)i * m + k) * J + j] = h[i];
    double gk = g[k * J + j];
    g[(k + 1) * J + j] = -s * gk;
    g[k * J + j] = c * gk;
    res[j] = fabs(g[(k + 1) * J + j]);
}

// Givens step k for every member
__global__ void k_givens(double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                         double* __restrict__ g, const double* __restrict__ hcol, const double* __restrict__ hn,
                         double* __restrict__ res, int k, int m, int J) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    givens_step(H, cs, sn, g, hcol + j, J, hn[j], res, k, m, J, j);
}

// One Gram-Schmidt pass with the norm from the dot products, one workgroup per
// member j: hcol[i J + j] = sum_b partial[(i J + j) nblk + b] for i <= k + 1 (per
// value the order of k_reduce: strided lane sums, then a butterfly), where rows
// i <= k are h = V^T w and row k + 1 is |w|^2; then hn[j] = sqrt(|w|^2 - sum_i
// h_i^2) (0 if not positive) and the Givens step k of member j as k_givens
__global__ void __launch_bounds__(kBlock) k_reduce_pyth_givens(const double* __restrict__ partial, int nblk,
                                                               double* __restrict__ hcol, double* __restrict__ hn,
                                                               double* __restrict__ H, double* __restrict__ cs,
                                                               double* __restrict__ sn, double* __restrict__ g,
                                                               double* __restrict__ res, double* __restrict__ clamps,
                                                               int k, int m, int J) {
    __shared__ double hs[kMaxRestart + 2];
    const int j = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i <= k + 1; i += kBlock / 64) {
        double sum = 0.0;
        for (int bk = lane; bk < nblk; bk += 64) sum += partial[((int64_t)i * J + j) * nblk + bk];
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (lane == 0) {
            hs[i] = sum;
            hcol[i * J + j] = sum;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s2 = 0.0;
    for (int i = 0; i <= k; ++i) s2 += hs[i] * hs[i];
    const double ww = hs[k + 1];   // |w|^2
    const double d = ww - s2;
    // |w|^2 - |h|^2 cancels once w lies almost in the span of the basis; a
    // difference that is not positive leaves the new vector zero (the member's
    // Krylov space is exhausted for this cycle).  That is right when the member
    // has converged and wrong when FP32 orthogonality noise caused it, so each
    // such event with w nonzero is counted.
    double hnj = 0.0;
    if (d > 0.0) hnj = sqrt(d);
    else if (ww > 0.0) clamps[j] += 1.0;
    hn[j] = hnj;
    givens_step(H, cs, sn, g, hs, 1, hnj, res, k, m, J, j);
}

// back substitution H(0:kd,0:kd) y = g(0:kd) per member
__global__ void k_lsq(const double* __restrict__ H, const double* __restrict__ g, double* __restrict__ y, int kd, int m,
                      int J) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    for (int i = kd - 1; i >= 0; --i) {
        double s = g[i * J + j];
        for (int c = i + 1; c < kd; ++c) s -= H[((int64_t)i * m + c) * J + j] * y[c * J + j];
        y[i * J + j] = s / H[((int64_t)i * m + i) * J + j];
    }
}

// weighted column sums for the pressure mean: partial[j * nblk + b] = sum_k w_k p[k,j]
__global__ void __launch_bounds__(kBlock) k_wsum(const double* __restrict__ p, const double* __restrict__ w, int64_t n,
                                                 int J, int CW, double* __restrict__ partial) {
    __shared__ double red[kBlock];
    const ColMap c = colmap(CW, 1, J);
    double acc = 0.0;
    if (c.ok)
        for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG)
            acc += w[r] * p[r * J + c.jb];
    double sv = block_colsum(acc, c, red, CW);
    if (c.ty == 0 && c.ok) partial[(int64_t)c.jb * gridDim.x + blockIdx.x] = sv;
}

__global__ void __launch_bounds__(kBlock) k_sub_mean(double* __restrict__ p, const double* __restrict__ sums,
                                                     double inv_area, int64_t n, int J) {
    int64_t idx = ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    for (; idx < n * J; idx += (int64_t)gridDim.x * kBlock) p[idx] -= sums[idx % J] * inv_area;
}

__global__ void k_fill64(double* __restrict__ a, int64_t n, double v) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_add_vec(double* __restrict__ a, const double* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

inline unsigned ew_grid(int64_t tot) {
    int64_t g = (tot + kBlock - 1) / kBlock;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 8192);
}

// launch shape of the column-reduction kernels for (n x J) blocks with VEC members per thread
struct RedShape {
    int CW, VEC, nblk;
    dim3 grid;
};

inline RedShape red_shape(int64_t n, int J, int vec_max) {
    RedShape s;
    s.VEC = 1;
    for (int v = vec_max; v > 1; v >>= 1)
        if (J % v == 0) {
            s.VEC = v;
            break;
        }
    int cols = J / s.VEC;
    int tiles = 1;
    if (cols <= kBlock) {
        s.CW = cols;
    } else {
        s.CW = 64;
        tiles = (cols + 63) / 64;
    }
    int RG = kBlock / s.CW;
    int64_t need = (n + RG - 1) / RG;
    s.nblk = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(need, 1));
    s.grid = dim3(s.nblk, tiles);
    return s;
}

inline unsigned reduce_grid(int64_t width) { return (unsigned)((width + (kBlock / 64) - 1) / (kBlock / 64)); }

#define LAUNCH_CHECK()                                     \
    do {                                                   \
        hipError_t e_ = hipGetLastError();                 \
        if (e_ != hipSuccess) {                            \
            set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
            return MHD_EHIP;                               \
        }                                                  \
    } while (0)

// ------------------------------------------------------------------ kernel timer
struct KTimer {
    bool on = false;
    int op = MHD_TUNE_SADDLE;   // the operator whose launches are timed
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    double ms = 0.0;
    int64_t launches = 0;
    double nJ32 = 0.0, nJ64 = 0.0;
};
KTimer g_timer;

hipError_t timer_fold() {
    for (size_t i = 0; i + 1 < g_timer.used; i += 2) {
        hipError_t e = hipEventSynchronize(g_timer.pool[i + 1]);
        if (e != hipSuccess) return e;
        float t = 0.f;
        e = hipEventElapsedTime(&t, g_timer.pool[i], g_timer.pool[i + 1]);
        if (e != hipSuccess) return e;
        g_timer.ms += t;
    }
    g_timer.used = 0;
    return hipSuccess;
}

// While t_ev0 is set, launch_k records the kernel's own start and end into
// (t_ev0, t_ev1) with the dispatch packet (the SpMM timer of the diagnostics).
thread_local hipEvent_t t_ev0 = nullptr, t_ev1 = nullptr;

// arms (t_ev0, t_ev1) for the next launch on st when the timer is on and st is
// not being captured; returns whether it did
bool timer_begin(hipStream_t st, int op) {
    if (!g_timer.on || g_timer.op != op) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    if (g_timer.used + 2 > g_timer.pool.size()) (void)timer_fold();
    if (g_timer.used + 2 > g_timer.pool.size()) return false;
    t_ev0 = g_timer.pool[g_timer.used++];
    t_ev1 = g_timer.pool[g_timer.used++];
    return true;
}

// vector width of the node-row fast path for J members (0: use the generic kernels)
inline int fast_vec(int J, int maxvec) {
    for (int v = maxvec; v >= 1; v >>= 1)
        if (J % (32 * v) == 0) return v;
    return 0;
}

inline dim3 node_grid(int64_t units, int J, int vec) { return dim3((unsigned)((units + 3) / 4), J / (32 * vec)); }

// runtime VEC -> compile-time dispatch (4 members per thread for FP32, 2 for FP64)
template <typename T, typename F>
mhd_status with_vec(int vec, F f) {
    if constexpr (sizeof(T) == 4) {
        if (vec == 4) return f(std::integral_constant<int, 4>{});
    }
    if (vec == 2) return f(std::integral_constant<int, 2>{});
    return f(std::integral_constant<int, 1>{});
}

inline RedShape cap_blocks(RedShape rs, int cap) {
    if (rs.nblk > cap) {
        rs.nblk = cap;
        rs.grid.x = cap;
    }
    return rs;
}

// ------------------------------------------------------------------ node-row kernel plans (autotuned)
// A plan picks, for one operator on one (mesh, J, word size), either the
// LDS-staged kernels (tile: square row tiles of 8, 12 or 16 half-steps; nw
// wavefronts per workgroup) or the gather kernels with vec members per lane per
// load (1, 2 or 4) and g units per wavefront (1, 2 or 4 batched gathers; 0 for
// one unit per wavefront with per-entry CSR loads).  vec == 0 selects the
// generic kernels (J not a multiple of 32).  Every candidate performs the same
// floating-point operations in the same order per member, so the choice changes
// the speed, not the result.
struct NodePlan {
    int vec = 0;
    int g = 0;
    int tile = 0;   // > 0: LDS-staged kernels on the tiling of this shape id
    int nw = 4;     // wavefronts per workgroup of the LDS-staged kernels
    int deep = 0;   // 1: pipelined gather kernels with g units per wavefront;
                    // 2: paired-row kernels with g units per wavefront
};

struct PlanRec {
    NodePlan p;
    float us = 0.f;
};

struct PlanKey {
    int64_t nP2, nP1, nnzA, nnzB;
    int J, word, op;
    bool operator<(const PlanKey& o) const {
        return std::tie(nP2, nP1, nnzA, nnzB, J, word, op) < std::tie(o.nP2, o.nP1, o.nnzA, o.nnzB, o.J, o.word, o.op);
    }
};

std::mutex g_plan_mu;
std::map<PlanKey, PlanRec> g_plans;

PlanKey plan_key(const DevMesh& m, int J, int word, int op) {
    return PlanKey{m.nP2, m.nP1, m.nnzA, m.nnzB, J, word, op};
}

inline int word_max_vec(int word) { return word == 4 ? 4 : 2; }

NodePlan default_plan(const DevMesh& m, int J, int word) {
    NodePlan p;
    p.vec = fast_vec(J, word_max_vec(word));
    p.g = (p.vec && m.max_row <= kMaxRowBatched) ? 1 : 0;
    return p;
}

NodePlan get_plan(const DevMesh& m, int J, int word, int op) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(plan_key(m, J, word, op));
    return it != g_plans.end() ? it->second.p : default_plan(m, J, word);
}

// vector loads need 16-byte aligned block bases; otherwise one member per lane
inline NodePlan align_plan(NodePlan p, bool aligned) {
    if (!aligned) {
        p.tile = 0;
        if (p.vec > 1) p.vec = 1;
    }
    return p;
}

// ------------------------------------------------------------------ row tilings (built on demand)
std::mutex g_tiling_mu;

int max_lds_bytes() {
    static int lim = -1;
    if (lim < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        lim = v;
    }
    return lim;
}

// builds and uploads the tiling of shape id on first use (host synchronous: not under capture)
mhd_status ensure_tiling(DevMesh& m, int id) {
    if (id < 1 || id > kTileShapes) return MHD_OK;
    std::lock_guard<std::mutex> lk(g_tiling_mu);
    if (m.tiling[id]) return MHD_OK;
    HostTiling h;
    build_tiling(m.host, tile_edge(id), tile_edge(id), h);
    auto* d = new (std::nothrow) DevTiling;
    if (!d) return MHD_ENOMEM;
    d->tx = h.tx;
    d->ty = h.ty;
    d->ntiles = h.ntiles;
    d->max_s2 = h.max_s2;
    d->max_s1 = h.max_s1;
    d->max_r2 = h.max_r2;
    d->max_r1 = h.max_r1;
    auto up = [&](int32_t** p, const std::vector<int32_t>& v) -> mhd_status {
        const size_t bytes = std::max<size_t>(v.size() * sizeof(int32_t), 256);
        hipError_t e = dev_malloc((void**)p, bytes);
        if (e == hipSuccess) {
            m.allocs.push_back(*p);
            if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            set_error(std::string("tiling upload: ") + hipGetErrorString(e));
            return MHD_ENOMEM;
        }
        return MHD_OK;
    };
    mhd_status rc = MHD_OK;
    if (!rc) rc = up(&d->r2_ptr, h.r2_ptr);
    if (!rc) rc = up(&d->r2, h.r2);
    if (!rc) rc = up(&d->r2_self, h.r2_self);
    if (!rc) rc = up(&d->r1_ptr, h.r1_ptr);
    if (!rc) rc = up(&d->r1, h.r1);
    if (!rc) rc = up(&d->r1_self, h.r1_self);
    if (!rc) rc = up(&d->s2_ptr, h.s2_ptr);
    if (!rc) rc = up(&d->s2, h.s2);
    if (!rc) rc = up(&d->s1_ptr, h.s1_ptr);
    if (!rc) rc = up(&d->s1, h.s1);
    if (!rc) rc = up(&d->a_loc, h.a_loc);
    if (!rc) rc = up(&d->bt_loc, h.bt_loc);
    if (!rc) rc = up(&d->b_loc, h.b_loc);
    if (!rc) rc = up(&d->ta_rp, h.ta_rp);
    if (!rc) rc = up(&d->ta_loc, h.ta_loc);
    if (!rc) rc = up(&d->ta_gp, h.ta_gp);
    if (!rc) rc = up(&d->tbt_rp, h.tbt_rp);
    if (!rc) rc = up(&d->tbt_loc, h.tbt_loc);
    if (!rc) rc = up(&d->tbt_gp, h.tbt_gp);
    if (!rc) rc = up(&d->tb_rp, h.tb_rp);
    if (!rc) rc = up(&d->tb_loc, h.tb_loc);
    if (!rc) rc = up(&d->tb_gp, h.tb_gp);
    d->max_ea = h.max_ea;
    d->max_ebt = h.max_ebt;
    d->max_eb = h.max_eb;
    if (rc) {
        delete d;
        return rc;
    }
    m.tiling[id] = d;
    return MHD_OK;
}

// builds and uploads the row-per-lane tiling of shape id on first use (host
// synchronous: not under capture); B and B^T entries are packed with their values
mhd_status ensure_ell(DevMesh& m, int id) {
    if (id < 1 || id > kEllShapes) return MHD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tiling_mu);
    if (m.ell[id]) return MHD_OK;
    HostEll h;
    build_ell(m.host, ell_tx(id), ell_ty(id), ell_m(id), h);
    const size_t nent = h.loc.size();
    std::vector<float> bt32(2 * (size_t)m.nnzBt), b32(2 * (size_t)m.nnzB);
    MHD_HIP(hipMemcpy(bt32.data(), m.valBt32, sizeof(float) * bt32.size(), hipMemcpyDeviceToHost));
    MHD_HIP(hipMemcpy(b32.data(), m.valB32, sizeof(float) * b32.size(), hipMemcpyDeviceToHost));
    auto bits = [](float f) {
        int32_t b;
        std::memcpy(&b, &f, 4);
        return b;
    };
    std::vector<int4> bm(nent);
    std::vector<int2> am(nent);
    std::vector<int32_t> posA((size_t)m.nnzA, -1);
    for (size_t e = 0; e < nent; ++e) {
        bm[e] = make_int4(h.loc[e], 0, 0, 0);
        am[e] = make_int2(h.loc[e], 0);
    }
    for (size_t b = 0; b < h.blk.size() / 8; ++b) {
        const int32_t* bd = &h.blk[8 * b];
        const int kind = bd[0], K1 = bd[2], K2 = bd[3], e1 = bd[4], e2 = bd[5];
        for (int e = e1; e < e1 + 64 * K1; ++e) {
            const int g = h.gp[e];
            if (g < 0) continue;
            if (kind == 0) {
                posA[g] = e;
            } else {
                bm[e].y = bits(b32[2 * (size_t)g]);
                bm[e].z = bits(b32[2 * (size_t)g + 1]);
            }
        }
        for (int e = e2; e < e2 + 64 * K2; ++e) {
            const int g = h.gp[e];
            if (g < 0) continue;
            bm[e].y = bits(bt32[2 * (size_t)g]);
            bm[e].z = bits(bt32[2 * (size_t)g + 1]);
        }
    }
    for (int32_t q : posA)
        if (q < 0) {
            set_error("row-per-lane tiling: an A entry has no slot");
            return MHD_EINVAL;
        }
    auto* d = new (std::nothrow) DevEll;
    if (!d) return MHD_ENOMEM;
    d->tx = h.tx;
    d->ty = h.ty;
    d->m = h.m;
    d->ntiles = h.ntiles;
    d->max_lds = h.max_lds;
    d->max_lds1 = h.max_lds1;
    d->max_lds2 = h.max_lds2;
    d->max_blocks = h.max_blocks;
    d->max_blocks2 = h.max_blocks2;
    d->max_k = h.max_k;
    d->nent = (int64_t)nent;
    auto up = [&](auto** p, const auto& v) -> mhd_status {
        const size_t bytes = std::max<size_t>(v.size() * sizeof(v[0]), 256);
        hipError_t e = dev_malloc((void**)p, bytes);
        if (e == hipSuccess) {
            m.allocs.push_back(*p);
            if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            set_error(std::string("row-per-lane tiling upload: ") + hipGetErrorString(e));
            return MHD_ENOMEM;
        }
        return MHD_OK;
    };
    mhd_status rc = MHD_OK;
    if (!rc) rc = up(&d->tile, h.tile);
    if (!rc) rc = up(&d->s2, h.s2);
    if (!rc) rc = up(&d->s1, h.s1);
    if (!rc) rc = up(&d->blk, h.blk);
    if (!rc) rc = up(&d->rows, h.rows);
    if (!rc) rc = up(&d->self, h.self);
    if (!rc) rc = up(&d->bm, bm);
    if (!rc) rc = up(&d->am0, am);
    if (!rc) rc = up(&d->posA, posA);
    if (rc) {
        delete d;
        return rc;
    }
    m.ell[id] = d;
    return MHD_OK;
}

// the operator's packed A entries for tiling id (allocated and filled on first
// use; later assemblies refresh them while a plan uses the tiling)
mhd_status ensure_ell_values(DevShared& S, int id, hipStream_t st) {
    mhd_status rc = ensure_ell(*S.mesh, id);
    if (rc) return rc;
    if (S.ellA[id]) return MHD_OK;
    const DevEll& t = *S.mesh->ell[id];
    int2* p = nullptr;
    const size_t bytes = sizeof(int2) * (size_t)std::max<int64_t>(t.nent, 64);
    MHD_HIP(dev_malloc((void**)&p, bytes));
    S.allocs.push_back(p);
    MHD_HIP(hipMemcpyAsync(p, t.am0, sizeof(int2) * (size_t)t.nent, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_ell_scatter, dim3((unsigned)((S.mesh->nnzA + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       S.valA32, t.posA, p, S.mesh->nnzA);
    MHD_HIP(hipGetLastError());
    MHD_HIP(hipStreamSynchronize(st));
    S.ellA[id] = p;
    return MHD_OK;
}

// as ensure_ell_values, and later assemblies keep the values current
mhd_status use_ell(DevShared& S, int id, hipStream_t st) {
    mhd_status rc = ensure_ell_values(S, id, st);
    if (rc) return rc;
    if (!S.ell_live[id]) {
        // values may be stale if assemblies ran while the tiling was unused
        hipLaunchKernelGGL(k_ell_scatter, dim3((unsigned)((S.mesh->nnzA + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           S.valA32, S.mesh->ell[id]->posA, S.ellA[id], S.mesh->nnzA);
        MHD_HIP(hipGetLastError());
        S.ell_live[id] = true;
    }
    return MHD_OK;
}

// shape code of the public interface: tx * 100 + ty, plus 10000 for 8 members per workgroup
inline int ell_code(int id) { return ell_tx(id) * 100 + ell_ty(id) + (ell_m(id) == 8 ? 10000 : 0); }
inline int ell_id(int code) {
    for (int id = 1; id <= kEllShapes; ++id)
        if (ell_code(id) == code) return id;
    return 0;
}

bool ell_usable(const DevShared& S, int id, int J) {
    if (id < 1 || id > kEllShapes || S.transposed || J % ell_m(id) || !S.ellA[id] || !S.mesh->ell[id]) return false;
    const DevEll& t = *S.mesh->ell[id];
    return t.max_blocks <= 8 && t.max_blocks2 <= 8 && t.max_lds + 16 <= max_lds_bytes();
}

}  // namespace

hipError_t scatter_ell_values(DevShared& S, hipStream_t s) {
    for (int id = 1; id <= kEllShapes; ++id) {
        if (!S.ellA[id] || !S.ell_live[id] || !S.mesh->ell[id]) continue;
        hipLaunchKernelGGL(k_ell_scatter, dim3((unsigned)((S.mesh->nnzA + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           S.valA32, S.mesh->ell[id]->posA, S.ellA[id], S.mesh->nnzA);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {

// Wave order of the paired-row and batched SpMM with g units per wavefront: the wavefronts
// of P2 units and of P1 units sorted by the P2 index of their first node, so
// that the divergence rows of a region run right after its velocity rows and
// find the velocity members they gather in L2.  Built once per mesh and g.
mhd_status ensure_pair_sched(DevMesh& m, int g) {
    if (g != 1 && g != 2 && g != 4 && g != 8) return MHD_OK;
    std::lock_guard<std::mutex> lk(g_tiling_mu);
    if (m.pair_sched[g]) return MHD_OK;
    const HostMesh& h = m.host;
    std::vector<int32_t> p2_of_p1(m.nP1, 0);
    for (int i = 0; i < m.nP2; ++i)
        if (h.p1_of_p2[i] >= 0) p2_of_p1[h.p1_of_p2[i]] = i;
    std::vector<std::pair<int64_t, int32_t>> waves;   // (key, entry)
    for (int u = 0; u < m.nP2; u += g) waves.push_back({2 * (int64_t)u, u});
    for (int k = 0; k < m.nP1; k += g) waves.push_back({2 * (int64_t)p2_of_p1[k] + 1, -(k + 1)});
    std::sort(waves.begin(), waves.end());
    std::vector<int32_t> sched(waves.size());
    for (size_t i = 0; i < waves.size(); ++i) sched[i] = waves[i].second;
    int32_t* d = nullptr;
    hipError_t e = dev_malloc((void**)&d, sched.size() * sizeof(int32_t));
    if (e == hipSuccess) {
        m.allocs.push_back(d);
        e = hipMemcpy(d, sched.data(), sched.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        set_error(std::string("pair schedule upload: ") + hipGetErrorString(e));
        return MHD_ENOMEM;
    }
    m.pair_sched[g] = d;
    return MHD_OK;
}

inline TileView tile_view(const DevTiling& t) {
    return TileView{t.r2_ptr, t.r2, t.r2_self, t.r1_ptr, t.r1, t.r1_self, t.s2_ptr, t.s2, t.s1_ptr, t.s1,
                    t.a_loc, t.bt_loc, t.b_loc};
}

// dynamic LDS of the staged kernels: SpMM and Jacobi first / later sweeps
inline size_t lds_bytes(const DevTiling& t, int op, int word, int vec) {
    const size_t jt = (size_t)kTileJ * vec * word;
    if (op == MHD_TUNE_JACOBI_FIRST) return (size_t)t.max_s1 * jt;
    if (op == MHD_TUNE_JACOBI) return (size_t)t.max_s2 * 2 * jt;
    return ((size_t)t.max_s2 * 2 + t.max_s1) * jt;
}

// LDS-staged kernels with staged entries (plan deep == 3): node values plus the
// tile's entries (value and 4-byte local column)
inline size_t lds_bytes_ent(const DevTiling& t, int op, int word, int vec) {
    const size_t x = lds_bytes(t, op, word, vec);
    if (op == MHD_TUNE_JACOBI_FIRST) return x + (size_t)t.max_ebt * (2 * word + 4);
    if (op == MHD_TUNE_JACOBI) return x + (size_t)t.max_ea * (word + 4);
    return x + (size_t)t.max_ea * (word + 4) + ((size_t)t.max_ebt + t.max_eb) * (2 * word + 4);
}

inline size_t plan_lds_bytes(const DevTiling& t, int op, int word, int vec, int deep) {
    return deep == 3 ? lds_bytes_ent(t, op, word, vec) : lds_bytes(t, op, word, vec);
}

inline TileEnt tile_ent(const DevTiling& t) {
    return TileEnt{t.ta_rp, t.ta_loc, t.ta_gp, t.tbt_rp, t.tbt_loc, t.tbt_gp, t.tb_rp, t.tb_loc, t.tb_gp};
}
inline TileDims tile_dims(const DevTiling& t) { return TileDims{t.max_s2, t.max_s1, t.max_ea, t.max_ebt, t.max_eb}; }

// LDS-staged kernels: members per lane the word size admits for J
inline bool lds_vec_ok(int J, int word, int vec) {
    return (vec == 1 || (vec == 2 && word == 4)) && J % (kTileJ * vec) == 0;
}

// each wavefront keeps the metadata of its rows in one register (<= 64 rows)
inline bool tile_fits(const DevTiling& t, int nw) { return t.max_r2 <= 64 * nw && t.max_r1 <= 64 * nw; }

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename F>
mhd_status with_g(int g, F f) {
    switch (g) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        default: return f(std::integral_constant<int, 0>{});
    }
}

template <typename F>
mhd_status with_gd(int g, F f) {
    switch (g) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return f(std::integral_constant<int, 1>{});
    }
}

// rows short enough for the pipelined kernels
inline bool deep_ok(const DevMesh& m) { return m.max_row <= kDeepA && m.max_row_bt <= kDeepBt; }

// paired-row kernels: J a multiple of 16 members per lane-load, short rows
// rows longer than kPairRow go in chunks (Scott-Vogelius meshes); Taylor-Hood rows fit one
inline bool pair_ok(const DevMesh& m, int J, int word) { return J % (256 / word) == 0; }

template <typename F>
mhd_status with_gp(int g, F f) {
    return g == 8 ? f(std::integral_constant<int, 8>{}) : f(std::integral_constant<int, 4>{});
}

inline dim3 group_grid(int64_t units, int J, int vec, int g) {
    const int64_t per = (int64_t)(kBlock / 64) * g;
    return dim3((unsigned)((units + per - 1) / per), J / (32 * vec));
}


template <typename K, typename... Args>
void launch_k(K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t st, Args... args) {
    if (t_ev0)
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, st, t_ev0, t_ev1, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
}

// y = S x (MODE 0) or y = b - S x (MODE 1) with plan p
template <typename T, int MODE>
mhd_status launch_saddle_plan(NodePlan p, DevShared& S, const T* x, const T* b, T* y, int J, hipStream_t st) {
    DevMesh& m = *S.mesh;
    const int64_t units = (int64_t)m.nP2 + m.nP1;
    if (p.deep == 6) {
        if constexpr (sizeof(T) == 4 && MODE == 0) {
            if (ell_usable(S, p.tile, J)) {
                const DevEll& t = *m.ell[p.tile];
                const int MS = J / t.m;
                const EllView E{t.tile, t.s2, t.s1, t.blk, t.rows, t.self, S.ellA[p.tile], t.bm};
                const dim3 grid((unsigned)((int64_t)t.ntiles * MS));
                const size_t lds = (size_t)t.max_lds + 16;   // + the slot of the staging overrun
                auto go = [&](auto kern, int threads) -> mhd_status {
                    MHD_HIP(allow_lds(kern, lds));
                    launch_k(kern, grid, dim3(threads), lds, st, E, Vals<float>::dp(m), x, y, m.nP2, J, MS);
                    LAUNCH_CHECK();
                    return MHD_OK;
                };
                auto by_waves = [&](auto Mc) -> mhd_status {
                    constexpr int MM = decltype(Mc)::value;
                    if (t.max_blocks <= 2) return go(k_saddle_e<MM, 2>, 128);
                    if (t.max_blocks <= 4) return go(k_saddle_e<MM, 4>, 256);
                    if (t.max_blocks <= 5) return go(k_saddle_e<MM, 5>, 320);
                    return go(k_saddle_e<MM, 8>, 512);
                };
                return t.m == 8 ? by_waves(std::integral_constant<int, 8>{}) : by_waves(std::integral_constant<int, 16>{});
            }
        }
        p = default_plan(m, J, sizeof(T));
    }
    if (p.tile > 0 && m.tiling[p.tile] && lds_vec_ok(J, sizeof(T), p.vec) && tile_fits(*m.tiling[p.tile], p.nw)) {
        const DevTiling& tl = *m.tiling[p.tile];
        const int MT = J / (kTileJ * p.vec);
        const size_t lds = plan_lds_bytes(tl, MHD_TUNE_SADDLE, sizeof(T), p.vec, p.deep);
        const dim3 grid((unsigned)((int64_t)tl.ntiles * MT));
        if (p.deep == 3 && deep_ok(m)) {
            auto go3 = [&](auto kern, int threads) -> mhd_status {
                MHD_HIP(allow_lds(kern, lds));
                launch_k(kern, grid, dim3(threads), lds, st, tile_view(tl), tile_ent(tl), tile_dims(tl), Vals<T>::A(S),
                         Vals<T>::Bt(S), Vals<T>::B(S), Vals<T>::dp(m), x, b, y, m.nP2, J, MT);
                LAUNCH_CHECK();
                return MHD_OK;
            };
            if constexpr (sizeof(T) == 4) {
                if (p.vec == 2)
                    return p.nw == 8 ? go3(k_saddle_t<T, 2, MODE, 8>, 512) : go3(k_saddle_t<T, 2, MODE, 4>, 256);
            }
            return p.nw == 8 ? go3(k_saddle_t<T, 1, MODE, 8>, 512) : go3(k_saddle_t<T, 1, MODE, 4>, 256);
        }
        auto go = [&](auto kern, int threads) -> mhd_status {
            MHD_HIP(allow_lds(kern, lds));
            launch_k(kern, grid, dim3(threads), lds, st, tile_view(tl), m.A_rowptr, Vals<T>::A(S),
                               m.Bt_rowptr, Vals<T>::Bt(S), m.B_rowptr, Vals<T>::B(S), Vals<T>::dp(m), x, b, y, m.nP2,
                               J, MT, tl.max_s2);
            LAUNCH_CHECK();
            return MHD_OK;
        };
        if constexpr (sizeof(T) == 4) {
            if (p.vec == 2) return p.nw == 8 ? go(k_saddle_lds<T, 2, MODE, 8>, 512) : go(k_saddle_lds<T, 2, MODE, 4>, 256);
        }
        return p.nw == 8 ? go(k_saddle_lds<T, 1, MODE, 8>, 512) : go(k_saddle_lds<T, 1, MODE, 4>, 256);
    }
    if (p.tile > 0) p = default_plan(m, J, sizeof(T));
    if (p.deep == 2 && pair_ok(m, J, sizeof(T))) {
        return with_gp(p.g, [&](auto Gc) -> mhd_status {
            constexpr int GG = decltype(Gc)::value;
            const int wP2 = (m.nP2 + GG - 1) / GG, wP1 = (m.nP1 + GG - 1) / GG;
            const dim3 grid((unsigned)((wP2 + wP1 + 3) / 4), J / (256 / (int)sizeof(T)));
            launch_k(k_saddle_h<T, MODE, GG>, grid, dim3(kBlock), 0, st, m.A_rowptr, m.A_col, Vals<T>::A(S),
                     m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S), m.B_rowptr, m.B_col, Vals<T>::B(S), Vals<T>::dp(m), x, b,
                     y, m.nP2, m.nP1, J, wP2, (const int32_t*)m.pair_sched[GG]);
            LAUNCH_CHECK();
            return MHD_OK;
        });
    }
    if (p.deep == 1 && p.vec && deep_ok(m)) {
        return with_vec<T>(p.vec, [&](auto V) -> mhd_status {
            constexpr int VV = decltype(V)::value;
            return with_gd(p.g, [&](auto Gc) -> mhd_status {
                constexpr int GG = decltype(Gc)::value;
                launch_k(k_saddle_p<T, VV, MODE, GG>, group_grid(units, J, VV, GG), dim3(kBlock), 0, st,
                                   m.A_rowptr, m.A_col, Vals<T>::A(S), m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S),
                                   m.B_rowptr, m.B_col, Vals<T>::B(S), Vals<T>::dp(m), x, b, y, m.nP2, m.nP1, J);
                LAUNCH_CHECK();
                return MHD_OK;
            });
        });
    }
    if (p.deep) p = default_plan(m, J, sizeof(T));
    if (p.vec == 0) {
        const int JP = pick_jp(J);
        launch_k(k_saddle<T, MODE>, dim3(grid_for(units, JP)), dim3(kBlock), 0, st, m.A_rowptr, m.A_col,
                           Vals<T>::A(S), m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S), m.B_rowptr, m.B_col, Vals<T>::B(S),
                           Vals<T>::dp(m), x, b, y, m.nP2, m.nP1, J, JP);
        LAUNCH_CHECK();
        return MHD_OK;
    }
    return with_vec<T>(p.vec, [&](auto V) -> mhd_status {
        constexpr int VV = decltype(V)::value;
        return with_g(p.g, [&](auto Gc) -> mhd_status {
            constexpr int GG = decltype(Gc)::value;
            if constexpr (GG == 0) {
                launch_k(k_saddle_v<T, VV, MODE>, node_grid(units, J, VV), dim3(kBlock), 0, st,
                                   m.A_rowptr, m.A_col, Vals<T>::A(S), m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S),
                                   m.B_rowptr, m.B_col, Vals<T>::B(S), Vals<T>::dp(m), x, b, y, m.nP2, m.nP1, J);
            } else {
                const int32_t* sched = m.pair_sched[GG];
                const int64_t nw = sched ? (m.nP2 + GG - 1) / GG + (m.nP1 + GG - 1) / GG : (units + GG - 1) / GG;
                const dim3 grid((unsigned)((nw + kBlock / 64 - 1) / (kBlock / 64)), J / (32 * VV));
                launch_k(k_saddle_g<T, VV, MODE, GG>, grid, dim3(kBlock), 0, st, m.A_rowptr, m.A_col, Vals<T>::A(S),
                         m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S), m.B_rowptr, m.B_col, Vals<T>::B(S), Vals<T>::dp(m), x,
                         b, y, m.nP2, m.nP1, J, sched);
            }
            LAUNCH_CHECK();
            return MHD_OK;
        });
    });
}

// velocity-block Jacobi with plan p.  FIRST: t = r_u - B^T z_p, zo = w D^-1 t
// (in = r_u); else zo = z + w D^-1 (t - A z).
template <typename T, bool FIRST>
mhd_status launch_velo_plan(NodePlan p, DevShared& S, const T* in, const T* zp, T* t, const T* z, T* zo, int J,
                            hipStream_t st, T omega) {
    if (p.deep == 6) {
        if constexpr (sizeof(T) == 4) {
            if (ell_usable(S, p.tile, J)) {
                const DevEll& tl = *S.mesh->ell[p.tile];
                const int MS = J / tl.m;
                const EllView E{tl.tile, tl.s2, tl.s1, tl.blk, tl.rows, tl.self, S.ellA[p.tile], tl.bm};
                const dim3 grid((unsigned)((int64_t)tl.ntiles * MS));
                const size_t lds = (size_t)(FIRST ? tl.max_lds1 : tl.max_lds2) + 16;
                auto go = [&](auto kern, int threads) -> mhd_status {
                    MHD_HIP(allow_lds(kern, lds));
                    launch_k(kern, grid, dim3(threads), lds, st, E, Vals<float>::dA(S), in, zp, t, z, zo, J, MS, omega);
                    LAUNCH_CHECK();
                    return MHD_OK;
                };
                auto by_waves = [&](auto Mc) -> mhd_status {
                    constexpr int MM = decltype(Mc)::value;
                    if (tl.max_blocks2 <= 2) return go(k_velo_e<MM, FIRST, 2>, 128);
                    if (tl.max_blocks2 <= 4) return go(k_velo_e<MM, FIRST, 4>, 256);
                    return go(k_velo_e<MM, FIRST, 8>, 512);
                };
                return tl.m == 8 ? by_waves(std::integral_constant<int, 8>{}) : by_waves(std::integral_constant<int, 16>{});
            }
        }
        p = default_plan(*S.mesh, J, sizeof(T));
    }
    DevMesh& m = *S.mesh;
    const int32_t* rp = FIRST ? m.Bt_rowptr : m.A_rowptr;
    const int32_t* col = FIRST ? m.Bt_col : m.A_col;
    const T* val = FIRST ? Vals<T>::Bt(S) : Vals<T>::A(S);
    if (p.tile > 0 && m.tiling[p.tile] && lds_vec_ok(J, sizeof(T), p.vec) && tile_fits(*m.tiling[p.tile], p.nw)) {
        const DevTiling& tl = *m.tiling[p.tile];
        const int MT = J / (kTileJ * p.vec);
        const size_t lds =
            plan_lds_bytes(tl, FIRST ? MHD_TUNE_JACOBI_FIRST : MHD_TUNE_JACOBI, sizeof(T), p.vec, p.deep);
        const dim3 grid((unsigned)((int64_t)tl.ntiles * MT));
        if (p.deep == 3 && deep_ok(m)) {
            auto go3 = [&](auto kern, int threads) -> mhd_status {
                MHD_HIP(allow_lds(kern, lds));
                launch_k(kern, grid, dim3(threads), lds, st, tile_view(tl), tile_ent(tl), tile_dims(tl), val,
                                   Vals<T>::dA(S), in, zp, t, z, zo, J, MT, omega);
                LAUNCH_CHECK();
                return MHD_OK;
            };
            if constexpr (sizeof(T) == 4) {
                if (p.vec == 2)
                    return p.nw == 8 ? go3(k_velo_t<T, 2, FIRST, 8>, 512) : go3(k_velo_t<T, 2, FIRST, 4>, 256);
            }
            return p.nw == 8 ? go3(k_velo_t<T, 1, FIRST, 8>, 512) : go3(k_velo_t<T, 1, FIRST, 4>, 256);
        }
        auto go = [&](auto kern, int threads) -> mhd_status {
            MHD_HIP(allow_lds(kern, lds));
            launch_k(kern, grid, dim3(threads), lds, st, tile_view(tl), rp, val, Vals<T>::dA(S), in, zp, t,
                               z, zo, J, MT, omega);
            LAUNCH_CHECK();
            return MHD_OK;
        };
        if constexpr (sizeof(T) == 4) {
            if (p.vec == 2) return p.nw == 8 ? go(k_velo_lds<T, 2, FIRST, 8>, 512) : go(k_velo_lds<T, 2, FIRST, 4>, 256);
        }
        return p.nw == 8 ? go(k_velo_lds<T, 1, FIRST, 8>, 512) : go(k_velo_lds<T, 1, FIRST, 4>, 256);
    }
    if (p.tile > 0) p = default_plan(m, J, sizeof(T));
    if (p.deep == 2 && pair_ok(m, J, sizeof(T))) {
        return with_gp(p.g, [&](auto Gc) -> mhd_status {
            constexpr int GG = decltype(Gc)::value;
            const int w = (m.nP2 + GG - 1) / GG;
            const dim3 grid((unsigned)((w + 3) / 4), J / (256 / (int)sizeof(T)));
            launch_k(k_velo_h<T, FIRST, GG>, grid, dim3(kBlock), 0, st, rp, col, val, Vals<T>::dA(S), in, zp, t, z,
                     zo, m.nP2, J, omega);
            LAUNCH_CHECK();
            return MHD_OK;
        });
    }
    if (p.deep == 1 && p.vec && deep_ok(m)) {
        return with_vec<T>(p.vec, [&](auto V) -> mhd_status {
            constexpr int VV = decltype(V)::value;
            return with_gd(p.g, [&](auto Gc) -> mhd_status {
                constexpr int GG = decltype(Gc)::value;
                launch_k(k_velo_p<T, VV, FIRST, GG>, group_grid(m.nP2, J, VV, GG), dim3(kBlock), 0, st,
                                   rp, col, val, Vals<T>::dA(S), in, zp, t, z, zo, m.nP2, J, omega);
                LAUNCH_CHECK();
                return MHD_OK;
            });
        });
    }
    if (p.deep) p = default_plan(m, J, sizeof(T));
    if (p.vec == 0) {
        const int JP = pick_jp(J);
        if (FIRST)
            launch_k(k_velo_first<T>, dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, st, rp, col, val,
                               Vals<T>::dA(S), in, zp, t, zo, m.nP2, J, JP, omega);
        else
            launch_k(k_velo_sweep<T>, dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, st, rp, col, val,
                               Vals<T>::dA(S), (const T*)t, z, zo, m.nP2, J, JP, omega);
        LAUNCH_CHECK();
        return MHD_OK;
    }
    return with_vec<T>(p.vec, [&](auto V) -> mhd_status {
        constexpr int VV = decltype(V)::value;
        return with_g(p.g, [&](auto Gc) -> mhd_status {
            constexpr int GG = decltype(Gc)::value;
            if constexpr (GG == 0) {
                launch_k(k_velo_v<T, VV, FIRST>, node_grid(m.nP2, J, VV), dim3(kBlock), 0, st, rp, col,
                                   val, Vals<T>::dA(S), in, zp, t, z, zo, m.nP2, J, omega);
            } else {
                launch_k(k_velo_g<T, VV, FIRST, GG>, group_grid(m.nP2, J, VV, GG), dim3(kBlock), 0, st,
                                   rp, col, val, Vals<T>::dA(S), in, zp, t, z, zo, m.nP2, J, omega);
            }
            LAUNCH_CHECK();
            return MHD_OK;
        });
    });
}

// Times every candidate plan of one operator on the handle's workspace buffers
// (contents irrelevant: zeroed first) and records the fastest.  Synchronises st.
template <typename T>
mhd_status tune_op(DevShared& S, int J, int op, hipStream_t st, std::vector<mhd_tune_entry>* rep) {
    DevMesh& m = *S.mesh;
    const int word = (int)sizeof(T);
    std::vector<NodePlan> cands;
    for (int v = word_max_vec(word); v >= 1; v >>= 1) {
        if (J % (32 * v)) continue;
        cands.push_back(NodePlan{v, 0, 0, 4, 0});
        if (m.max_row <= kMaxRowBatched)
            for (int g : {1, 2, 4}) {
                mhd_status rc = ensure_pair_sched(m, g);
                if (rc) return rc;
                cands.push_back(NodePlan{v, g, 0, 4, 0});
            }
        if (deep_ok(m))
            for (int g : {1, 2, 4, 8}) cands.push_back(NodePlan{v, g, 0, 4, 1});
    }
    if (pair_ok(m, J, word))
        for (int g : {4, 8}) {
            mhd_status rc = ensure_pair_sched(m, g);
            if (rc) return rc;
            cands.push_back(NodePlan{16 / word, g, 0, 4, 2});
        }
    for (int v : {2, 1}) {
        if (!lds_vec_ok(J, word, v) || sv_mesh(m)) continue;
        for (int id = 1; id <= kTileShapes; ++id) {
            mhd_status rc = ensure_tiling(m, id);
            if (rc) return rc;
            for (int dp : {0, 3}) {
                if (dp == 3 && !deep_ok(m)) continue;
                if (plan_lds_bytes(*m.tiling[id], op, word, v, dp) > (size_t)max_lds_bytes()) continue;
                for (int nw : {4, 8})
                    if (tile_fits(*m.tiling[id], nw)) cands.push_back(NodePlan{v, 0, id, nw, dp});
            }
        }
    }
    if (word == 4 && op != MHD_TUNE_RESIDUAL && J % 8 == 0 && !S.transposed && !sv_mesh(m))
        for (int id = 1; id <= kEllShapes; ++id) {
            mhd_status rc = ensure_ell_values(S, id, st);
            if (rc) return rc;
            if (ell_usable(S, id, J)) cands.push_back(NodePlan{4, 0, id, 0, 6});
        }
    PlanRec best;
    if (!cands.empty()) {
        T* x = (T*)S.gw.zbuf;
        T* y = (T*)S.gw.wbuf;
        T* t = (T*)S.gw.tbuf;
        T* b = (T*)S.gw.r64;
        const size_t bytes = sizeof(T) * (size_t)m.n * J;
        MHD_HIP(hipMemsetAsync(x, 0, bytes, st));
        MHD_HIP(hipMemsetAsync(t, 0, bytes, st));
        MHD_HIP(hipMemsetAsync(b, 0, bytes, st));
        const T* xp = x + 2 * (int64_t)m.nP2 * J;
        auto run = [&](const NodePlan& p) -> mhd_status {
            switch (op) {
                case MHD_TUNE_SADDLE: return launch_saddle_plan<T, 0>(p, S, x, nullptr, y, J, st);
                case MHD_TUNE_RESIDUAL:
                    if constexpr (sizeof(T) == 8) return launch_saddle_plan<T, 1>(p, S, x, b, y, J, st);
                    return MHD_EINVAL;
                case MHD_TUNE_JACOBI_FIRST: return launch_velo_plan<T, true>(p, S, x, xp, t, nullptr, y, J, st, (T)0.7);
                default: return launch_velo_plan<T, false>(p, S, nullptr, nullptr, t, x, y, J, st, (T)0.7);
            }
        };
        hipEvent_t e0 = nullptr, e1 = nullptr;
        MHD_HIP(hipEventCreate(&e0));
        MHD_HIP(hipEventCreate(&e1));
        mhd_status rc = MHD_OK;
        best.us = 1e30f;
        std::vector<float> times(cands.size(), 0.f);
        constexpr int kReps = 10;
        for (size_t c = 0; c < cands.size() && rc == MHD_OK; ++c) {
            if (run(cands[c]) != MHD_OK) {   // warm-up; a shape the device refuses is skipped
                (void)hipGetLastError();
                times[c] = -1.f;
                continue;
            }
            if (hipEventRecord(e0, st) != hipSuccess) rc = MHD_EHIP;
            for (int r = 0; r < kReps && rc == MHD_OK; ++r) rc = run(cands[c]);
            if (rc == MHD_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = MHD_EHIP;
            float ms = 0.f;
            if (rc == MHD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MHD_EHIP;
            times[c] = 1000.f * ms / kReps;
            if (rc == MHD_OK && times[c] < best.us) best = PlanRec{cands[c], times[c]};
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) {
            if (rc == MHD_EHIP) set_error("autotune: HIP event failure");
            return rc;
        }
        if (rep)
            for (size_t c = 0; c < cands.size(); ++c) {
                const NodePlan& q = cands[c];
                const bool same = q.tile == best.p.tile && q.vec == best.p.vec && q.deep == best.p.deep &&
                                  (q.tile ? q.nw == best.p.nw : q.g == best.p.g);
                rep->push_back(mhd_tune_entry{op, word, J, q.vec, q.tile ? 0 : q.g, q.deep,
                                              q.tile ? (q.deep == 6 ? ell_code(q.tile) : tile_edge(q.tile)) : 0,
                                              q.tile ? q.nw : 0, times[c], same ? 1 : 0});
            }
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[plan_key(m, J, word, op)] = best;
    return MHD_OK;
}

bool plan_cached(const DevMesh& m, int J, int word, int op) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    return g_plans.count(plan_key(m, J, word, op)) != 0;
}

}  // namespace

// The plan one operator runs with for (mesh, J, word size): the table entry
// (chosen = 1) or the default plan (chosen = 0), in the autotuner's report form.
mhd_status query_plan(DevShared& S, int J, int precision, int op, mhd_tune_entry* out) {
    DevMesh& m = *S.mesh;
    if (op < MHD_TUNE_SADDLE || op > MHD_TUNE_JACOBI) {
        set_error("mhd_ens_get_plan: unknown operator");
        return MHD_EINVAL;
    }
    const int word = (op == MHD_TUNE_RESIDUAL || precision == MHD_FP64) ? 8 : 4;
    PlanRec r{default_plan(m, J, word), -1.f};
    bool tuned = false;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(plan_key(m, J, word, op));
        if (it != g_plans.end()) {
            r = it->second;
            tuned = true;
        }
    }
    const NodePlan& q = r.p;
    *out = mhd_tune_entry{op, word, J, q.vec, q.tile ? 0 : q.g, q.deep,
                          q.tile ? (q.deep == 6 ? ell_code(q.tile) : tile_edge(q.tile)) : 0, q.tile ? q.nw : 0, r.us,
                          tuned ? 1 : 0};
    return MHD_OK;
}

// Tunes the node-row operators a solve of this precision uses (inner SpMM and
// Jacobi sweeps in the inner word size, FP64 residual).  Without force, only
// missing plans are tuned.  Does nothing (and returns MHD_OK) while st is being
// captured: the cached or default plans are used then.
// Pins the plan of one operator for (mesh, J, word size), replacing the tuned one.
mhd_status set_plan(DevShared& S, int J, int precision, int op, int vec, int group, int deep, int tile, int waves) {
    DevMesh& m = *S.mesh;
    const int word = (precision == MHD_FP32_IR && op != MHD_TUNE_RESIDUAL) ? 4 : 8;
    if (op < MHD_TUNE_SADDLE || op > MHD_TUNE_JACOBI) {
        set_error("mhd_ens_set_plan: unknown operator");
        return MHD_EINVAL;
    }
    if (sv_mesh(m) && (tile || deep == 3 || deep == 6)) {
        set_error("mhd_ens_set_plan: row tiles are built on the half-step grid of Taylor-Hood meshes");
        return MHD_EINVAL;
    }
    if (deep == 6) {
        const int id = ell_id(tile);
        if (word != 4 || op == MHD_TUNE_RESIDUAL || !id || J % ell_m(id)) {
            set_error("mhd_ens_set_plan: row-per-lane tiles (deep 6) are an FP32 plan (SpMM and Jacobi sweeps) with "
                      "tile 1616, 3208 or 1608 (16 members per workgroup, J a multiple of 16) or 11616, 13208 or "
                      "11608 (8 members, J a multiple of 8)");
            return MHD_EINVAL;
        }
        mhd_status rc = use_ell(S, id, nullptr);
        if (rc) return rc;
        MHD_HIP(hipStreamSynchronize(nullptr));
        if (!ell_usable(S, id, J)) {
            set_error("mhd_ens_set_plan: tile needs more LDS or row blocks than a workgroup may use");
            return MHD_EINVAL;
        }
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[plan_key(m, J, word, op)] = PlanRec{NodePlan{4, 0, id, 0, 6}, 0.f};
        return MHD_OK;
    }
    if (deep == 2) {
        if (tile || !(group == 4 || group == 8) || !pair_ok(m, J, word)) {
            set_error("mhd_ens_set_plan: paired rows need group 4 or 8 and J a multiple of 256 / word size");
            return MHD_EINVAL;
        }
        mhd_status rc = ensure_pair_sched(m, group);
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[plan_key(m, J, word, op)] = PlanRec{NodePlan{16 / word, group, 0, 4, 2}, 0.f};
        return MHD_OK;
    }
    if (!(vec == 0 || vec == 1 || vec == 2 || (vec == 4 && word == 4)) || (vec && J % (32 * vec))) {
        set_error("mhd_ens_set_plan: vec must be 0 or 1, 2 (4 for FP32) with J a multiple of 32 vec");
        return MHD_EINVAL;
    }
    if (deep == 3 && !tile) {
        set_error("mhd_ens_set_plan: staged entries (deep 3) need an LDS tile");
        return MHD_EINVAL;
    }
    if (tile) {
        // checked below
    } else if (deep == 1) {
        if (!vec || !(group == 1 || group == 2 || group == 4 || group == 8) || !deep_ok(m)) {
            set_error("mhd_ens_set_plan: pipelined gathers need vec > 0, group 1, 2, 4 or 8 and rows of <= 24 (B^T: "
                      "8) entries");
            return MHD_EINVAL;
        }
    } else if (deep != 0) {
        set_error("mhd_ens_set_plan: deep must be 0, 1, 2, 3 or 6");
        return MHD_EINVAL;
    } else if (!(group == 0 || group == 1 || group == 2 || group == 4) || (group && m.max_row > kMaxRowBatched)) {
        set_error("mhd_ens_set_plan: group must be 0, 1, 2 or 4 (batched gathers need rows of <= 56 entries)");
        return MHD_EINVAL;
    }
    int id = 0;
    if (tile) {
        for (int k = 1; k <= kTileShapes; ++k)
            if (tile_edge(k) == tile) id = k;
        if (!id || !(waves == 4 || waves == 8) || !lds_vec_ok(J, word, vec) || !(deep == 0 || deep == 3) ||
            (deep == 3 && !deep_ok(m))) {
            set_error("mhd_ens_set_plan: tile must be 0, 8, 12 or 16 with waves 4 or 8, vec 1 (or 2 for FP32) and J a "
                      "multiple of 32 vec");
            return MHD_EINVAL;
        }
        mhd_status rc = ensure_tiling(m, id);
        if (rc) return rc;
        if (plan_lds_bytes(*m.tiling[id], op, word, vec, deep) > (size_t)max_lds_bytes() ||
            !tile_fits(*m.tiling[id], waves)) {
            set_error("mhd_ens_set_plan: tile needs more LDS or rows per wavefront than a workgroup may use");
            return MHD_EINVAL;
        }
    }
    if (vec && !id && deep == 0 && group) {
        mhd_status rc = ensure_pair_sched(m, group);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[plan_key(m, J, word, op)] = PlanRec{NodePlan{vec, (vec && !id) ? group : 0, id, waves, vec ? deep : 0}, 0.f};
    return MHD_OK;
}

mhd_status autotune(DevShared& S, int J, int precision, hipStream_t st, bool force, std::vector<mhd_tune_entry>* rep) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MHD_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return MHD_OK;
    DevMesh& m = *S.mesh;
    const int word = precision == MHD_FP32_IR ? 4 : 8;
    mhd_status rc;
    for (int op : {MHD_TUNE_SADDLE, MHD_TUNE_JACOBI_FIRST, MHD_TUNE_JACOBI}) {
        if (!force && plan_cached(m, J, word, op)) continue;
        rc = word == 4 ? tune_op<float>(S, J, op, st, rep) : tune_op<double>(S, J, op, st, rep);
        if (rc) return rc;
    }
    if (force || !plan_cached(m, J, 8, MHD_TUNE_RESIDUAL))
        if ((rc = tune_op<double>(S, J, MHD_TUNE_RESIDUAL, st, rep))) return rc;
    // plans are shared by meshes of equal size: make sure this mesh holds the tilings they use
    for (int op : {MHD_TUNE_SADDLE, MHD_TUNE_JACOBI_FIRST, MHD_TUNE_JACOBI, MHD_TUNE_RESIDUAL}) {
        const NodePlan p = get_plan(m, J, op == MHD_TUNE_RESIDUAL ? 8 : word, op);
        if (p.deep == 6) {
            if ((rc = use_ell(S, p.tile, st))) return rc;
        } else if (p.tile && (rc = ensure_tiling(*S.mesh, p.tile))) {
            return rc;
        }
        if ((p.deep == 2 || (p.deep == 0 && p.tile == 0)) && (rc = ensure_pair_sched(*S.mesh, p.g))) return rc;
    }
    return MHD_OK;
}

namespace {

// ------------------------------------------------------------------ host-side operators
template <typename T>
struct Ops {
    DevShared& S;
    int J;
    hipStream_t st;
    int JP;

    NodePlan p_saddle, p_first, p_sweep;   // autotuned node-row kernels for this (mesh, J, word size)
    bool fused_mg = true;                  // V-cycle levels as their two fused operators
    int mg_cycles = 1;                     // V-cycles per Schur-part application (1 or 2)
    int mg_post = 0;                       // extra post-smoothing sweeps on the finest level

    Ops(DevShared& s, int j, hipStream_t stream) : S(s), J(j), st(stream), JP(pick_jp(j)) {
        const int word = (int)sizeof(T);
        p_saddle = get_plan(*S.mesh, J, word, MHD_TUNE_SADDLE);
        p_first = get_plan(*S.mesh, J, word, MHD_TUNE_JACOBI_FIRST);
        p_sweep = get_plan(*S.mesh, J, word, MHD_TUNE_JACOBI);
    }

    mhd_status saddle(const T* x, T* y) {
        const bool timed = timer_begin(st, MHD_TUNE_SADDLE);
        const bool aligned = (((uintptr_t)x | (uintptr_t)y) % 16) == 0;
        mhd_status rc = launch_saddle_plan<T, 0>(align_plan(p_saddle, aligned), S, x, nullptr, y, J, st);
        t_ev0 = t_ev1 = nullptr;
        if (rc) return rc;
        if (timed) {
            g_timer.launches++;
            (sizeof(T) == 4 ? g_timer.nJ32 : g_timer.nJ64) += (double)J;
        }
        return MHD_OK;
    }

    // the packed-row kernels apply (J a multiple of 256 bytes of members, rows of <= 32 entries)
    bool packed(const DevCSR<double>& c) const { return J % (256 / (int)sizeof(T)) == 0 && c.max_row <= 32; }

    template <int MODE>
    mhd_status csr(const DevCSR<double>& c, const T* dinv, const T* x, const T* b, T* y, T omega, int pin = -1) {
        constexpr int MJ = 256 / (int)sizeof(T);
        if (J % MJ == 0) {
            // 16 lanes per row, four rows per wavefront, 16-byte member loads; rows
            // of more than 16 entries in chunks of 16 (faster than 32 lanes per row
            // for the 17-entry vertex-grid rows as for the 66-entry discontinuous
            // ones, with the same operations in the same order)
            const int64_t waves = (c.nrows + 3) / 4;
            hipLaunchKernelGGL((k_mg<T, MODE, 16>), dim3((unsigned)((waves + 3) / 4), J / MJ), dim3(kBlock), 0, st,
                               c.rowptr, c.col, Vals<T>::csr(c), dinv, x, b, y, (int)c.nrows, J, omega, pin);
        } else if constexpr (MODE == 6) {
            return MHD_EINVAL;   // callers check packed() first
        } else {
            hipLaunchKernelGGL((k_csr<T, MODE>), dim3(grid_for(c.nrows, JP)), dim3(kBlock), 0, st, c.rowptr, c.col,
                               Vals<T>::csr(c), dinv, x, b, y, c.nrows, J, JP, omega);
        }
        LAUNCH_CHECK();
        return MHD_OK;
    }

    // One V(2,2)-cycle with damped Jacobi smoothing on level l for L_l x = b.
    // Uses the level's buffers x, x2, r and the next level's b and x.  Returns
    // the buffer holding the result in *out.
    // dest (level 0, no schur): the buffer the last sweep writes instead of the level's x2
    mhd_status vcycle(int l, const T* b, T** out, T* schur = nullptr, int pin = -1, T* dest = nullptr) {
        const DevLevel& Lv = S.levels[l];
        T* x = (T*)S.gw.mg_x[l];
        mhd_status rc;
        if (l + 1 == (int)S.levels.size()) {
            if constexpr (std::is_same<T, float>::value) {
                if (J % 16 == 0) {
                    hipLaunchKernelGGL(k_dense_mf, dim3((Lv.n + 15) / 16, J / 16), dim3(kDenseWaves * 64), 0, st,
                                       Lv.cinv32, b, x, Lv.n, Lv.ld32, J);
                    LAUNCH_CHECK();
                    *out = x;
                    return MHD_OK;
                }
            }
            T* part = (T*)S.gw.dense_part;
            hipLaunchKernelGGL((k_dense_part<T>), dim3((Lv.n + 63) / 64, (J + 63) / 64, kDenseKS), dim3(kBlock), 0,
                               st, Vals<T>::cinv(Lv), b, part, Lv.n, Vals<T>::cinv_ld(Lv), J);
            LAUNCH_CHECK();
            const int64_t nJ = (int64_t)Lv.n * J;
            hipLaunchKernelGGL((k_dense_sum<T>), dim3((unsigned)((nJ + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                               (const T*)part, x, nJ);
            LAUNCH_CHECK();
            *out = x;
            return MHD_OK;
        }
        const T omega = (T)Lv.omega;
        T* x2 = (T*)S.gw.mg_x2[l];
        T* r = (T*)S.gw.mg_r[l];
        T* bc = (T*)S.gw.mg_b[l + 1];
        const T* dinv = Vals<T>::dinv(Lv);
        // x2 = x + w D^-1 (b - L x) with x = w D^-1 b: two sweeps from a zero guess in one pass
        if ((rc = csr<5>(Lv.L, dinv, nullptr, b, x2, omega))) return rc;
        const bool fuse = fused_mg && packed(Lv.L) && Lv.Dn.nnz > 0 && Lv.Dn.max_row <= 64 && Lv.Up.max_row <= 64;
        const int MJ = 256 / (int)sizeof(T);
        if (fuse) {   // bc = R (b - L x2) = [R | -R L] [b; x2]
            const dim3 gd((unsigned)(((Lv.Dn.nrows + 1) / 2 + 3) / 4), J / MJ);
            hipLaunchKernelGGL((k_mgf<T>), gd, dim3(kBlock), 0, st, Lv.Dn.rowptr, Lv.Dn.col, Vals<T>::csr(Lv.Dn), b,
                               (const T*)x2, (const T*)nullptr, Lv.n, Lv.n, bc, (int)Lv.Dn.nrows, J);
            LAUNCH_CHECK();
        } else {
            if ((rc = csr<2>(Lv.L, dinv, x2, b, r, omega))) return rc;        // r  = b - L x2
            if ((rc = csr<0>(Lv.R, dinv, r, nullptr, bc, omega))) return rc;  // bc = R r
        }
        T* xc = nullptr;
        if ((rc = vcycle(l + 1, bc, &xc))) return rc;
        if (fuse) {   // x = E (x2 + P xc) + w D^-1 b = [E | E P | w D^-1] [x2; xc; b]
            const dim3 gu((unsigned)(((Lv.Up.nrows + 1) / 2 + 3) / 4), J / MJ);
            hipLaunchKernelGGL((k_mgf<T>), gu, dim3(kBlock), 0, st, Lv.Up.rowptr, Lv.Up.col, Vals<T>::csr(Lv.Up),
                               (const T*)x2, (const T*)xc, b, Lv.n, S.levels[l + 1].n, x, (int)Lv.Up.nrows, J);
            LAUNCH_CHECK();
        } else {
            if ((rc = csr<1>(Lv.P, dinv, xc, nullptr, x2, omega))) return rc; // x2 += P xc
            if ((rc = csr<3>(Lv.L, dinv, x2, b, x, omega))) return rc;        // post-smoothing
        }
        if (l == 0)   // extra post-smoothing on the finest level (x -> x2 -> x ...)
            for (int q = 0; q < mg_post; ++q) {
                if ((rc = csr<3>(Lv.L, dinv, x, b, x2, omega))) return rc;
                std::swap(x, x2);
            }
        if (schur) {   // the last sweep writes the Schur part z_p directly
            if ((rc = csr<6>(Lv.L, dinv, x, b, schur, omega, pin))) return rc;
            *out = schur;
            return MHD_OK;
        }
        T* fin = dest ? dest : x2;
        if ((rc = csr<3>(Lv.L, dinv, x, b, fin, omega))) return rc;
        *out = fin;
        return MHD_OK;
    }

    // z = P^{-1} v (block upper-triangular preconditioner)
    mhd_status precond(const T* v, T* z, int sweeps, double omega_d) {
        DevMesh& m = *S.mesh;
        const int64_t off = 2 * (int64_t)m.nP2 * J;
        const T* vp = v + off;
        T* zp = z + off;
        mhd_status rc;
        T* xmg = nullptr;
        if (mg_cycles == 2 && S.levels.size() > 1 && (packed(S.levels[0].L) || sv_mesh(m))) {
            // two V-cycles: x1 = V(r_p), x2 = V(r_p - L x1), z_p = -(x1 + x2)
            T* x1 = (T*)S.gw.mg_y0;
            T* res = (T*)S.gw.mg_b[0];
            const DevLevel& L0 = S.levels[0];
            if ((rc = vcycle(0, vp, &xmg, nullptr, -1, x1))) return rc;   // the first cycle ends in x1
            if ((rc = csr<2>(L0.L, Vals<T>::dinv(L0), x1, vp, res, (T)kMgOmega))) return rc;
            if ((rc = vcycle(0, res, &xmg))) return rc;
            hipLaunchKernelGGL((k_schur2<T>), dim3(ew_grid((int64_t)m.nP1 * J)), dim3(kBlock), 0, st, (const T*)x1,
                               (const T*)xmg, vp, m.pin, zp, (int64_t)m.nP1, J);
            LAUNCH_CHECK();
        } else if (S.levels.size() > 1 && packed(S.levels[0].L)) {
            if ((rc = vcycle(0, vp, &xmg, zp, m.pin))) return rc;   // z_p written by the last smoothing sweep
        } else {
            if ((rc = vcycle(0, vp, &xmg))) return rc;
            hipLaunchKernelGGL((k_schur<T>), dim3(grid_for(m.nP1, JP)), dim3(kBlock), 0, st, xmg, vp, m.pin, zp,
                               m.nP1, J, JP);
            LAUNCH_CHECK();
        }
        const T omega = (T)omega_d;
        T* t = (T*)S.gw.tbuf;
        // ping-pong between z and z2buf, starting so that the last sweep writes z
        T* za = (sweeps % 2) ? z : (T*)S.gw.z2buf;
        T* zb = (sweeps % 2) ? (T*)S.gw.z2buf : z;
        const bool aligned = (((uintptr_t)v | (uintptr_t)z | (uintptr_t)t | (uintptr_t)zb) % 16) == 0;
        const NodePlan pf = align_plan(p_first, aligned), ps = align_plan(p_sweep, aligned);
        int s = 1;
        if (sweeps >= 2 && pf.deep == 2 && ps.deep == 2 && pair_ok(m, J, sizeof(T))) {
            // first sweep stores t only; the second forms z1 = w D^-1 t on the fly
            if ((rc = launch_velo_plan<T, true>(pf, S, v, zp, t, nullptr, nullptr, J, st, omega))) return rc;
            T* z2 = ((sweeps - 2) % 2 == 0) ? z : (T*)S.gw.z2buf;   // so that the last sweep writes z
            rc = with_gp(ps.g, [&](auto Gc) -> mhd_status {
                constexpr int GG = decltype(Gc)::value;
                const int w = (m.nP2 + GG - 1) / GG;
                hipLaunchKernelGGL((k_velo_h2<T, GG>), dim3((unsigned)((w + 3) / 4), J / (256 / (int)sizeof(T))),
                                   dim3(kBlock), 0, st, m.A_rowptr, m.A_col, Vals<T>::A(S), Vals<T>::dA(S),
                                   (const T*)t, z2, m.nP2, J, omega);
                LAUNCH_CHECK();
                return MHD_OK;
            });
            if (rc) return rc;
            za = z2;
            zb = (z2 == z) ? (T*)S.gw.z2buf : z;
            s = 2;
        } else if ((rc = launch_velo_plan<T, true>(pf, S, v, zp, t, nullptr, za, J, st, omega))) {
            return rc;
        }
        for (; s < sweeps; ++s) {
            const bool timed = timer_begin(st, MHD_TUNE_JACOBI);
            rc = launch_velo_plan<T, false>(ps, S, nullptr, nullptr, t, za, zb, J, st, omega);
            t_ev0 = t_ev1 = nullptr;
            if (rc) return rc;
            if (timed) {
                g_timer.launches++;
                (sizeof(T) == 4 ? g_timer.nJ32 : g_timer.nJ64) += (double)J;
            }
            std::swap(za, zb);
        }
        if (za != z) {
            hipError_t e = hipMemcpyAsync(z, za, sizeof(T) * (size_t)2 * m.nP2 * J, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) {
                set_error(std::string("precond copy: ") + hipGetErrorString(e));
                return MHD_EHIP;
            }
        }
        return MHD_OK;
    }

    mhd_status colnorm(const double* a, double* out) {
        int64_t n = S.mesh->n;
        RedShape rs = red_shape(n, J, ((uintptr_t)a % 16 == 0) ? 2 : 1);
        rs = cap_blocks(rs, S.gw.nblk_cap);
        mhd_status rc = with_vec<double>(rs.VEC, [&](auto V) -> mhd_status {
            hipLaunchKernelGGL((k_colsq<decltype(V)::value>), rs.grid, dim3(kBlock), 0, st, a, n, J, rs.CW,
                               S.gw.partial);
            LAUNCH_CHECK();
            return MHD_OK;
        });
        if (rc) return rc;
        hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(J)), dim3(kBlock), 0, st, S.gw.partial, rs.nblk, (int64_t)J, out,
                           1);
        LAUNCH_CHECK();
        return MHD_OK;
    }
};

inline size_t slot_bytes(int64_t nrows, int Jmax) { return (((size_t)nrows * Jmax * sizeof(double)) + 255) & ~(size_t)255; }

template <typename T>
inline T* basis_ptr(DevShared& S, int i) {
    return (T*)((char*)S.gw.basis + (size_t)i * slot_bytes(S.gw.nrows, S.Jmax));
}

mhd_status sync_copy(double* host, const double* dev, int J, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(host, dev, sizeof(double) * J, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error(std::string("solver synchronisation: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    return MHD_OK;
}

// f(integral_constant<int, nb>) for nb = 1 ... 8
template <typename F>
mhd_status with_nb(int nb, F f) {
    switch (nb) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        default: return f(std::integral_constant<int, 8>{});
    }
}

// out = a / s (per column) with 16-byte loads where the shape allows, else elementwise
template <typename TI, typename TO>
mhd_status launch_scale_cols(const TI* a, const double* s, TO* out, int64_t n, int J, hipStream_t st) {
    constexpr int V = 16 / (int)sizeof(TI);
    const RedShape rs = red_shape(n, J, V);
    if (rs.VEC == V && ((uintptr_t)a | (uintptr_t)out) % 16 == 0) {
        const int RG = kBlock / rs.CW;
        const unsigned nb = (unsigned)std::min<int64_t>(8192, (n + RG - 1) / RG);
        hipLaunchKernelGGL((k_scale_cols_v<TI, TO, V>), dim3(nb, rs.grid.y), dim3(kBlock), 0, st, a, s, 1, out, n, J,
                           rs.CW);
    } else {
        hipLaunchKernelGGL((k_scale_cols<TI, TO>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, a, s, 1, out, n, J);
    }
    LAUNCH_CHECK();
    return MHD_OK;
}

template <typename T>
mhd_status gmres_solve(DevShared& S, const double* b, double* x, int J, const mhd_solver_opts& o,
                       mhd_solve_stats* stt, hipStream_t st, bool compact_ok = true);

__global__ void k_gather_cols(const double* __restrict__ src, double* __restrict__ dst,
                              const int32_t* __restrict__ idx, int64_t n, int J, int Jc) {
    for (int64_t q = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; q < n * Jc; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / Jc;
        dst[q] = src[r * J + idx[q - r * Jc]];
    }
}

__global__ void k_scatter_cols(const double* __restrict__ src, double* __restrict__ dst,
                               const int32_t* __restrict__ idx, int64_t n, int J, int Jc) {
    for (int64_t q = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; q < n * Jc; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / Jc;
        dst[r * J + idx[q - r * Jc]] = src[q];
    }
}

// Adaptive per-member solve once some members have met rtol: the remaining
// members' right-hand sides and iterates are gathered into a block of Jc < J
// columns, solved on (every kernel streams Jc columns; the converged iterates
// are left as they are), and scattered back; the statistics cover all J.
template <typename T>
mhd_status compacted_solve(DevShared& S, const double* b, double* x, int J, const std::vector<int32_t>& act,
                           const mhd_solver_opts& o, mhd_solve_stats* stt, hipStream_t st, int iters0, int cycles0,
                           const std::vector<int>& first_met) {
    GmresWork& G = S.gw;
    const int64_t n = S.mesh->n;
    const int Jc = (int)act.size();
    MHD_HIP(hipMemcpyAsync(G.cidx, act.data(), sizeof(int32_t) * Jc, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gather_cols, dim3(ew_grid(n * Jc)), dim3(kBlock), 0, st, b, G.cb, (const int32_t*)G.cidx, n,
                       J, Jc);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather_cols, dim3(ew_grid(n * Jc)), dim3(kBlock), 0, st, (const double*)x, G.cx,
                       (const int32_t*)G.cidx, n, J, Jc);
    LAUNCH_CHECK();
    MHD_HIP(hipStreamSynchronize(st));   // act is host memory that the copy reads
    mhd_solver_opts oc = o;
    oc.maxit = std::max(1, o.maxit - iters0);
    std::vector<double> rel_c(Jc);
    std::vector<int32_t> it_c(Jc);
    mhd_solve_stats sc{};
    sc.relres = rel_c.data();
    sc.member_iters = it_c.data();
    const mhd_status rc = gmres_solve<T>(S, G.cb, G.cx, Jc, oc, &sc, st, false);
    if (rc != MHD_OK && rc != MHD_ENOCONV) return rc;
    hipLaunchKernelGGL(k_scatter_cols, dim3(ew_grid(n * Jc)), dim3(kBlock), 0, st, (const double*)G.cx, x,
                       (const int32_t*)G.cidx, n, J, Jc);
    LAUNCH_CHECK();
    if (stt) {
        // final residuals of all J members
        Ops<double> ops(S, J, st);
        mhd_status r2;
        if ((r2 = saddle_residual64(S, b, x, G.r64, J, st))) return r2;
        if ((r2 = ops.colnorm(G.r64, G.beta))) return r2;
        if ((r2 = ops.colnorm(b, G.bnorm))) return r2;
        std::vector<double> hb(J), hn(J);
        MHD_HIP(hipMemcpyAsync(hb.data(), G.beta, sizeof(double) * J, hipMemcpyDeviceToHost, st));
        MHD_HIP(hipMemcpyAsync(hn.data(), G.bnorm, sizeof(double) * J, hipMemcpyDeviceToHost, st));
        MHD_HIP(hipStreamSynchronize(st));
        double mx = 0.0;
        int bad = 0;
        for (int j = 0; j < J; ++j) {
            const double r = hn[j] > 0 ? hb[j] / hn[j] : hb[j];
            if (!std::isfinite(r)) ++bad;
            else mx = std::max(mx, r);
            if (stt->relres) stt->relres[j] = r;
            if (stt->member_iters) stt->member_iters[j] = first_met[j] >= 0 ? first_met[j] : iters0;
        }
        for (int i = 0; i < Jc; ++i)
            if (stt->member_iters) stt->member_iters[act[i]] = iters0 + it_c[i];
        stt->iters = iters0 + sc.iters;
        stt->cycles = cycles0 + sc.cycles;
        stt->max_relres = bad ? NAN : mx;
        stt->converged = (rc == MHD_OK) ? 1 : 0;
        stt->nonfinite = bad;
        stt->min_block_rank = J;
        stt->norm_clamps = sc.norm_clamps;
        stt->compacted = Jc;
    }
    return rc;
}

// Gram-Schmidt norms taken as zero in the last solve on this handle (fused
// single pass), summed over members (synchronises; never called under capture)
int norm_clamp_count(GmresWork& G, int J, hipStream_t st) {
    std::vector<double> f(J, 0.0);
    if (hipMemcpyAsync(f.data(), G.res + 2 * J, sizeof(double) * J, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    double sum = 0.0;
    for (double v : f) sum += v;
    return (int)sum;
}

template <typename T>
mhd_status gmres_solve(DevShared& S, const double* b, double* x, int J, const mhd_solver_opts& o,
                       mhd_solve_stats* stt, hipStream_t st, bool compact_ok) {
    DevMesh& m = *S.mesh;
    GmresWork& G = S.gw;
    const int64_t n = m.n;
    const int mres = std::max(1, std::min(o.restart > 0 ? o.restart : G.restart, G.restart));
    const int check = std::max(1, o.check_every);
    const int sweeps = std::max(1, o.jacobi_sweeps);
    const double omega = o.jacobi_omega > 0 ? o.jacobi_omega : kJacobiOmega;
    Ops<T> ops(S, J, st);
    ops.fused_mg = o.mg_unfused == 0;
    ops.mg_cycles = o.mg_cycles == 2 ? 2 : 1;
    ops.mg_post = o.mg_post;
    RedShape rs = cap_blocks(red_shape(n, J, 16 / (int)sizeof(T)), G.nblk_cap);
    // cgs_passes: 1 or 2 classical passes with the norm taken directly, 3 one pass
    // with the norm from the dot products (fused kernels), 0 the default (one pass
    // for FP32 inner solves, two for FP64)
    const bool pyth = o.cgs_passes == 3;
    const int passes = pyth ? 1 : (o.cgs_passes > 0 ? o.cgs_passes : (sizeof(T) == 4 ? 1 : 2));
    const T* const* Vd = (const T* const*)G.dptrs;
    // FP32 solves keep z_k = P^-1 v_k (flexible form), saving one preconditioner
    // application per refinement cycle; FP64 solves recompute P^-1 (V y)
    const bool keepz = sizeof(T) == 4 && G.zbasis != nullptr;
    const T* const* Zd = (const T* const*)G.zptrs;
    const size_t zblk = (((size_t)n * S.Jmax * sizeof(float)) + 255) & ~(size_t)255;
    auto zslot = [&](int k) { return (T*)((char*)G.zbasis + (size_t)k * zblk); };
    double* hres = G.host_res;                 // pinned, 3 J doubles: residuals, beta, bnorm
    double* hbeta = G.host_res + J;
    double* hbn = G.host_res + 2 * J;
    double* hcol2 = G.hcol + (int64_t)(kMaxRestart + 1) * J;
    double* hn = G.res + J;
    mhd_status rc;
    // fixed schedule: fixed_cycles refinement cycles of mres inner iterations,
    // no host synchronisation (graph-capturable)
    const bool fixed = o.fixed_cycles > 0;
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(kBlock), 0, st, G.res + 2 * J, (int64_t)J, 0.0);
    LAUNCH_CHECK();
    if (!fixed) {
        if ((rc = ops.colnorm(b, G.bnorm))) return rc;
        if ((rc = sync_copy(hbn, G.bnorm, J, st))) return rc;
    }
    int iters = 0, cycles = 0;
    double maxrel = 0.0;
    bool conv = false;
    // inner iterations after which each member's true residual first met rtol
    std::vector<int> first_met(fixed ? 0 : J, -1);
    auto fill_stats = [&](bool ok, bool nonfinite) {
        if (!stt) return;
        stt->norm_clamps = fixed ? -1 : norm_clamp_count(G, J, st);
        stt->compacted = 0;
        stt->iters = iters;
        stt->cycles = cycles;
        stt->max_relres = fixed ? -1.0 : maxrel;
        stt->converged = fixed ? -1 : (ok ? 1 : 0);
        stt->min_block_rank = J;
        stt->nonfinite = 0;
        for (int j = 0; j < J; ++j) {
            double rel = fixed ? -1.0 : (hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j]);
            if (!fixed && !std::isfinite(rel)) ++stt->nonfinite;
            if (stt->relres) stt->relres[j] = rel;
            if (stt->member_iters) stt->member_iters[j] = (fixed || first_met[j] < 0) ? iters : first_met[j];
        }
        (void)nonfinite;
    };
    while (true) {
        // FP64 residual r = b - S x and its column norms
        if (fixed && cycles >= o.fixed_cycles) break;
        if ((rc = saddle_residual64(S, b, x, G.r64, J, st))) return rc;
        if ((rc = ops.colnorm(G.r64, G.beta))) return rc;
        if (!fixed) {
        if ((rc = sync_copy(hbeta, G.beta, J, st))) return rc;
        maxrel = 0.0;
        bool bad = false;
        for (int j = 0; j < J; ++j) {
            double rel = hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j];
            if (!std::isfinite(rel)) bad = true;
            maxrel = std::max(maxrel, rel);
        }
        for (int j = 0; j < J; ++j) {
            const double rel = hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j];
            if (first_met[j] < 0 && rel <= o.rtol) first_met[j] = iters;
        }
        if (bad) {
            set_error("mhd_ens_solve: non-finite residual");
            fill_stats(false, true);
            return MHD_ENOCONV;
        }
        if (maxrel <= o.rtol) {
            conv = true;
            break;
        }
        if (iters >= o.maxit) break;
        if (compact_ok && !o.keep_converged && G.cb) {
            // some members converged: the others continue as a compacted block
            std::vector<int32_t> act;
            for (int j = 0; j < J; ++j)
                if (!(first_met[j] >= 0)) act.push_back(j);
            if (!act.empty() && (int)act.size() < J)
                return compacted_solve<T>(S, b, x, J, act, o, stt, st, iters, cycles, first_met);
        }
        }
        // v0 = r / beta in the inner precision; g = beta e1
        if ((rc = launch_scale_cols<double, T>(G.r64, G.beta, basis_ptr<T>(S, 0), n, J, st))) return rc;
        hipLaunchKernelGGL(k_init_g, dim3((J + 255) / 256), dim3(256), 0, st, G.g, G.beta, mres + 1, J);
        LAUNCH_CHECK();
        int kd = 0;
        for (int k = 0; k < mres && (fixed || iters < o.maxit); ++k) {
            T* vk = basis_ptr<T>(S, k);
            T* z = keepz ? zslot(k) : (T*)G.zbuf;
            T* w = basis_ptr<T>(S, k + 1);
            if ((rc = ops.precond(vk, z, sweeps, omega))) return rc;
            if ((rc = ops.saddle(z, w))) return rc;
            if (pyth) {
                // one classical Gram-Schmidt pass: |w|^2 comes with the dot products,
                // h_{k+1,k} = sqrt(|w|^2 - |h|^2) (V orthonormal), and the update
                // stores v_{k+1} = (w - V h) / h_{k+1,k} directly; the last vector of
                // a cycle is never used, so its update is skipped
                for (int c0 = 0; c0 <= k; c0 += 8) {
                    const int nb = std::min(8, k + 1 - c0);
                    const bool last = c0 + nb == k + 1;
                    rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                        return with_nb(nb, [&](auto NBc) -> mhd_status {
                            constexpr int VV = decltype(V)::value, NN = decltype(NBc)::value;
                            if (last)
                                hipLaunchKernelGGL((k_dots<T, VV, NN, true>), rs.grid, dim3(kBlock), 0, st, Vd, c0,
                                                   (const T*)w, n, J, rs.CW, G.partial);
                            else
                                hipLaunchKernelGGL((k_dots<T, VV, NN, false>), rs.grid, dim3(kBlock), 0, st, Vd, c0,
                                                   (const T*)w, n, J, rs.CW, G.partial);
                            LAUNCH_CHECK();
                            return MHD_OK;
                        });
                    });
                    if (rc) return rc;
                }
                hipLaunchKernelGGL(k_reduce_pyth_givens, dim3(J), dim3(kBlock), 0, st, (const double*)G.partial,
                                   rs.nblk, G.hcol, hn, G.H, G.cs, G.sn, G.g, G.res, G.res + 2 * J, k, mres, J);
                LAUNCH_CHECK();
                for (int c0 = 0; c0 <= k && k + 1 < mres; c0 += 8) {
                    const int nb = std::min(8, k + 1 - c0);
                    const double* sc = c0 + nb == k + 1 ? (const double*)hn : nullptr;
                    rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                        return with_nb(nb, [&](auto NBc) -> mhd_status {
                            constexpr int VV = decltype(V)::value, NN = decltype(NBc)::value;
                            hipLaunchKernelGGL((k_update<T, VV, NN, false>), rs.grid, dim3(kBlock), 0, st, Vd, c0,
                                               (const double*)G.hcol, w, n, J, rs.CW, G.partial, 1, sc);
                            LAUNCH_CHECK();
                            return MHD_OK;
                        });
                    });
                    if (rc) return rc;
                }
            } else {
            // classical Gram-Schmidt with a re-orthogonalisation pass
            for (int pass = 0; pass < passes; ++pass) {
                double* hdst = pass ? hcol2 : G.hcol;
                for (int c0 = 0; c0 <= k; c0 += 8) {
                    const int nb = std::min(8, k + 1 - c0);
                    rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                        return with_nb(nb, [&](auto NBc) -> mhd_status {
                            hipLaunchKernelGGL((k_dots<T, decltype(V)::value, decltype(NBc)::value>), rs.grid,
                                               dim3(kBlock), 0, st, Vd, c0, (const T*)w, n, J, rs.CW, G.partial);
                            LAUNCH_CHECK();
                            return MHD_OK;
                        });
                    });
                    if (rc) return rc;
                }
                hipLaunchKernelGGL(k_reduce, dim3(reduce_grid((int64_t)(k + 1) * J)), dim3(kBlock), 0, st, G.partial,
                                   rs.nblk, (int64_t)(k + 1) * J, hdst, 0);
                LAUNCH_CHECK();
                for (int c0 = 0; c0 <= k; c0 += 8) {
                    const int nb = std::min(8, k + 1 - c0);
                    const bool last = c0 + nb == k + 1;
                    rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                        return with_nb(nb, [&](auto NBc) -> mhd_status {
                            constexpr int VV = decltype(V)::value, NN = decltype(NBc)::value;
                            // the last vector of a cycle is only needed for its norm
                            const int store = (k + 1 < mres || pass + 1 < passes) ? 1 : 0;
                            if (last)
                                hipLaunchKernelGGL((k_update<T, VV, NN, true>), rs.grid, dim3(kBlock), 0, st, Vd, c0,
                                                   (const double*)hdst, w, n, J, rs.CW, G.partial, store);
                            else
                                hipLaunchKernelGGL((k_update<T, VV, NN, false>), rs.grid, dim3(kBlock), 0, st, Vd, c0,
                                                   (const double*)hdst, w, n, J, rs.CW, G.partial);
                            LAUNCH_CHECK();
                            return MHD_OK;
                        });
                    });
                    if (rc) return rc;
                }
            }
            hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(J)), dim3(kBlock), 0, st, G.partial, rs.nblk, (int64_t)J, hn,
                               1);
            LAUNCH_CHECK();
            if (passes == 2) {   // h = h1 + h2 over the two passes
                hipLaunchKernelGGL(k_add_vec, dim3(((k + 1) * J + 255) / 256), dim3(256), 0, st, G.hcol,
                                   (const double*)hcol2, (int64_t)(k + 1) * J);
                LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_givens, dim3((J + 63) / 64), dim3(64), 0, st, G.H, G.cs, G.sn, G.g, G.hcol, hn,
                               G.res, k, mres, J);
            LAUNCH_CHECK();
            // v_{k+1} = w / h_{k+1,k}; the last vector of a cycle is never used
            if (k + 1 < mres)
                if ((rc = launch_scale_cols<T, T>(w, hn, w, n, J, st))) return rc;
            }
            ++iters;
            kd = k + 1;
            if (!fixed && (kd % check == 0 || kd == mres)) {
                if ((rc = sync_copy(hres, G.res, J, st))) return rc;
                bool done = true;
                for (int j = 0; j < J; ++j) {
                    double target = std::max(o.inner_rtol * hbeta[j], 0.5 * o.rtol * hbn[j]);
                    if (!(hres[j] <= target)) done = false;
                }
                if (done) break;
            }
        }
        // x += P^{-1} (V y), or with the preconditioned vectors kept, x += Z y (Z = P^-1 V)
        hipLaunchKernelGGL(k_lsq, dim3((J + 63) / 64), dim3(64), 0, st, G.H, G.g, G.y, kd, mres, J);
        LAUNCH_CHECK();
        T* u = (T*)G.wbuf;
        // with Z kept the last chunk adds its result to x directly (16-byte aligned x)
        const bool fuse_x = keepz && ((uintptr_t)x % 16) == 0;
        for (int c0 = 0; c0 < kd; c0 += 8) {
            const int nb = std::min(8, kd - c0);
            double* x64 = (fuse_x && c0 + nb == kd) ? x : nullptr;
            rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                return with_nb(nb, [&](auto NBc) -> mhd_status {
                    constexpr int VV = decltype(V)::value, NN = decltype(NBc)::value;
                    if (c0 == 0)
                        hipLaunchKernelGGL((k_combine<T, VV, NN, true>), rs.grid, dim3(kBlock), 0, st, keepz ? Zd : Vd,
                                           c0, (const double*)G.y, u, n, J, rs.CW, x64);
                    else
                        hipLaunchKernelGGL((k_combine<T, VV, NN, false>), rs.grid, dim3(kBlock), 0, st, keepz ? Zd : Vd,
                                           c0, (const double*)G.y, u, n, J, rs.CW, x64);
                    LAUNCH_CHECK();
                    return MHD_OK;
                });
            });
            if (rc) return rc;
        }
        if (!keepz) {
            if ((rc = ops.precond(u, (T*)G.zbuf, sweeps, omega))) return rc;
            hipLaunchKernelGGL((k_add_to64<T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, x, (const T*)G.zbuf, n * J);
            LAUNCH_CHECK();
        } else if (!fuse_x && kd > 0) {
            hipLaunchKernelGGL((k_add_to64<T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, x, (const T*)u, n * J);
            LAUNCH_CHECK();
        }
        ++cycles;
    }
    fill_stats(conv, false);
    if (fixed) return MHD_OK;
    if (!conv) {
        set_error("mhd_ens_solve: maxit reached before rtol (best iterate written)");
        return MHD_ENOCONV;
    }
    return MHD_OK;
}

// ------------------------------------------------------------------ block GMRES
// One Krylov space shared by the J right-hand sides (paper, Section 1: the
// shared matrix pairs naturally with block linear solvers): the basis grows by
// blocks V_k of up to J orthonormal columns, the block upper-Hessenberg H is
// built by block classical Gram-Schmidt with a second pass, and each new block
// is orthonormalised by a pivoted Cholesky QR whose small pivots deflate the
// directions that have become dependent (identical members, converged ones).
// Deflated columns are zero and stay zero through the linear preconditioner
// and the SpMM, so every kernel keeps the (n, J) block layout.

// Per-workgroup partials of the J x J product A^T B of two (n, J) blocks in
// FP64 (J = 16 TA): the workgroup's rows go through LDS 32 at a time and each
// thread owns a TA x TA tile of the product.  Layout of the partials as
// k_reduce expects: partial[(a J + b) nblk + workgroup].
template <typename T, int TA>
__global__ void __launch_bounds__(kBlock) k_bgram(const T* __restrict__ A, const T* __restrict__ B, int64_t n,
                                                  double* __restrict__ partial) {
    constexpr int J = 16 * TA;
    constexpr int RT = 32;
    __shared__ T sa[RT * J], sb[RT * J];
    const int t = threadIdx.x;
    const int a0 = (t / 16) * TA, b0 = (t % 16) * TA;
    double acc[TA][TA];
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int k = 0; k < TA; ++k) acc[i][k] = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
    for (int64_t rb = r0; rb < r1; rb += RT) {
        for (int q = t; q < RT * J; q += kBlock) {
            const int64_t row = rb + q / J;
            T va = 0, vb = 0;
            if (row < r1) {
                va = A[row * J + q % J];
                vb = B[row * J + q % J];
            }
            sa[q] = va;
            sb[q] = vb;
        }
        __syncthreads();
        for (int rr = 0; rr < RT; ++rr) {
            double xa[TA], xb[TA];
#pragma unroll
            for (int i = 0; i < TA; ++i) {
                xa[i] = (double)sa[rr * J + a0 + i];
                xb[i] = (double)sb[rr * J + b0 + i];
            }
#pragma unroll
            for (int i = 0; i < TA; ++i)
#pragma unroll
                for (int k = 0; k < TA; ++k) acc[i][k] += xa[i] * xb[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int k = 0; k < TA; ++k) partial[((int64_t)(a0 + i) * J + b0 + k) * gridDim.x + blockIdx.x] = acc[i][k];
}

// C (op)= A M for (n, J) blocks A, C and a J x J matrix M (FP64, staged in
// LDS): MODE 0 C = A M, 1 C -= A M, 2 C += A M.  Lanes over the J columns of a
// row; A's row is read by every lane of the row (one broadcast load per entry).
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_bmm(const T* __restrict__ A, const double* __restrict__ M,
                                                T* __restrict__ C, int64_t n, int J) {
    extern __shared__ double sm[];
    for (int q = threadIdx.x; q < J * J; q += kBlock) sm[q] = M[q];
    __syncthreads();
    const int rpb = kBlock / J;
    const int b = threadIdx.x % J, sub = threadIdx.x / J;
    if (sub >= rpb) return;
    for (int64_t row = (int64_t)blockIdx.x * rpb + sub; row < n; row += (int64_t)gridDim.x * rpb) {
        const T* ar = A + row * J;
        double acc = 0.0;
        for (int a = 0; a < J; ++a) acc += (double)ar[a] * sm[a * J + b];
        T* c = C + row * J + b;
        if (MODE == 0)
            *c = (T)acc;
        else if (MODE == 1)
            *c = (T)((double)*c - acc);
        else
            *c = (T)((double)*c + acc);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_convert(const double* __restrict__ a, T* __restrict__ out, int64_t tot) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < tot; i += (int64_t)gridDim.x * kBlock)
        out[i] = (T)a[i];
}

// Small dense algebra of the block solver on the host (FP64, row-major J x J).
struct BlockQR {
    int J = 0;
    // Pivoted Cholesky of a Gram matrix G = W^T W: W Pi = Q U with rank p (pivots
    // whose square falls below tol2 times the largest diagonal of G are
    // dropped).  Returns p; Minv (J x J) maps W to Q (Q = W Minv, columns >= p
    // zero) and C (J x J) has W = Q C (rows >= p zero).
    int factor(const std::vector<double>& G, double tol2, std::vector<double>& Minv, std::vector<double>& C) const {
        std::vector<double> A(G);
        std::vector<int> piv(J);
        for (int i = 0; i < J; ++i) piv[i] = i;
        double dmax = 0.0;
        for (int i = 0; i < J; ++i) dmax = std::max(dmax, A[(size_t)i * J + i]);
        std::vector<double> U((size_t)J * J, 0.0);   // rows in pivot order, columns in original order
        int p = 0;
        for (; p < J; ++p) {
            int best = -1;
            double bv = 0.0;
            for (int i = p; i < J; ++i) {
                const double d = A[(size_t)piv[i] * J + piv[i]];
                if (d > bv) {
                    bv = d;
                    best = i;
                }
            }
            if (best < 0 || !(bv > tol2 * dmax) || !(dmax > 0.0)) break;
            std::swap(piv[p], piv[best]);
            const int c = piv[p];
            const double r = std::sqrt(bv);
            U[(size_t)p * J + c] = r;
            for (int i = p + 1; i < J; ++i) U[(size_t)p * J + piv[i]] = A[(size_t)c * J + piv[i]] / r;
            for (int i = p + 1; i < J; ++i)
                for (int k = p + 1; k < J; ++k) {
                    const int a = piv[i], bb = piv[k];
                    A[(size_t)a * J + bb] -= U[(size_t)p * J + a] * U[(size_t)p * J + bb];
                }
        }
        C.assign((size_t)J * J, 0.0);
        for (int k = 0; k < p; ++k)
            for (int c = 0; c < J; ++c) C[(size_t)k * J + c] = U[(size_t)k * J + c];
        // Q = W[:, piv[0..p)] U11^-1 with U11[k][i] = U[k][piv[i]] upper triangular
        Minv.assign((size_t)J * J, 0.0);
        std::vector<double> inv((size_t)p * p, 0.0);
        for (int col = 0; col < p; ++col) {   // solve U11 x = e_col (back substitution)
            for (int i = p - 1; i >= 0; --i) {
                double v = (i == col) ? 1.0 : 0.0;
                for (int k = i + 1; k < p; ++k) v -= U[(size_t)i * J + piv[k]] * inv[(size_t)k * p + col];
                inv[(size_t)i * p + col] = v / U[(size_t)i * J + piv[i]];
            }
        }
        for (int i = 0; i < p; ++i)
            for (int k = 0; k < p; ++k) Minv[(size_t)piv[i] * J + k] = inv[(size_t)i * p + k];
        return p;
    }
};

// Least squares min || E1 C0 - Hb Y ||_F for the (m+1)J x mJ block Hessenberg
// Hb, updated one block column per Arnoldi step (the block form of GMRES's
// Givens updates): the new column block receives the Householder reflections
// of all earlier columns, then gets its own J reflections (each spans at most
// 2J rows, the column's nonzeros below its diagonal), which are applied to the
// right-hand side block too.  After step k the transformed right-hand side rows
// below the triangle give every member's least-squares residual.  Zero pivots
// (deflated directions) leave their Y rows 0.
struct BlockLSQ {
    int J = 0, mres = 0, cols = 0;
    std::vector<std::vector<double>> Wb;   // column block k: (k + 2) J rows x J columns, column-major
    std::vector<double> rhs;  // (mres + 1) J rows x J
    std::vector<double> vref; // per column: its reflector over rows c .. c + 2J - 1 (zero-padded)
    std::vector<double> vnorm;
    std::vector<char> dead;
    void reset(int J_, int mres_, const std::vector<double>& C0) {
        J = J_;
        mres = mres_;
        cols = 0;
        const size_t R = (size_t)(mres + 1) * J, C = (size_t)mres * J;
        // the column blocks and reflectors are written before they are read, so
        // they are not cleared; a block's storage is sized when it is added
        if ((int)Wb.size() < mres) Wb.resize(mres);
        rhs.assign(R * J, 0.0);
        for (int a = 0; a < J; ++a)
            for (int c = 0; c < J; ++c) rhs[(size_t)a * J + c] = C0[(size_t)a * J + c];
        vref.resize(C * 2 * J);
        vnorm.assign(C, 0.0);
        dead.assign(C, 0);
    }
    double& w(int r, int c) {
        const int k = c / J;
        return Wb[k][(size_t)(c - k * J) * (k + 2) * J + r];
    }
    // applies reflector q to columns [c0, c1) of W, or to the right-hand side if rhs_too
    void reflect(int q, int c0, int c1, bool to_rhs) {
        if (dead[q] || !(vnorm[q] > 0.0)) return;
        const int rows = (mres + 1) * J, last = std::min(rows, (q / J + 2) * J);
        const double* v = &vref[(size_t)q * 2 * J];
        const int len = last - q;
        for (int c = c0; c < c1; ++c) {
            double* x = &w(q, c);   // a column's rows are contiguous
            double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
            int r = 0;
            for (; r + 4 <= len; r += 4) {
                d0 += v[r] * x[r];
                d1 += v[r + 1] * x[r + 1];
                d2 += v[r + 2] * x[r + 2];
                d3 += v[r + 3] * x[r + 3];
            }
            for (; r < len; ++r) d0 += v[r] * x[r];
            const double d = 2.0 * ((d0 + d1) + (d2 + d3)) / vnorm[q];
            for (r = 0; r < len; ++r) x[r] -= d * v[r];
        }
        if (to_rhs)
            for (int k = 0; k < J; ++k) {
                double d = 0.0;
                for (int r = q; r < last; ++r) d += v[r - q] * rhs[(size_t)r * J + k];
                d = 2.0 * d / vnorm[q];
                for (int r = q; r < last; ++r) rhs[(size_t)r * J + k] -= d * v[r - q];
            }
    }
    // column block k: H[i * mres + k] for i <= k + 1 (J x J each, row-major)
    void add_block(int k, const std::vector<std::vector<double>>& H) {
        const int c0 = k * J, c1 = c0 + J;
        Wb[k].resize((size_t)(k + 2) * J * J);
        for (int i = 0; i <= k + 1; ++i) {
            const std::vector<double>& hb = H[(size_t)i * mres + k];
            for (int a = 0; a < J; ++a)
                for (int c = 0; c < J; ++c) w(i * J + a, c0 + c) = hb[(size_t)a * J + c];
        }
        for (int q = 0; q < c0; ++q) reflect(q, c0, c1, false);
        const int rows = (mres + 1) * J;
        for (int c = c0; c < c1; ++c) {
            const int last = std::min(rows, (c / J + 2) * J);
            double nrm = 0.0;
            for (int r = c; r < last; ++r) nrm += w(r, c) * w(r, c);
            nrm = std::sqrt(nrm);
            double* v = &vref[(size_t)c * 2 * J];
            if (!(nrm > 1e-300)) {
                dead[c] = 1;
                continue;
            }
            const double x0 = w(c, c);
            const double alpha = x0 >= 0 ? -nrm : nrm;
            for (int r = c; r < last; ++r) v[r - c] = w(r, c);
            v[0] -= alpha;
            double vv = 0.0;
            for (int r = c; r < last; ++r) vv += v[r - c] * v[r - c];
            vnorm[c] = vv;
            reflect(c, c, c1, true);
        }
        cols = c1;
    }
    // every member's least-squares residual after the blocks added so far
    void residuals(std::vector<double>& res) const {
        res.assign(J, 0.0);
        for (int r = cols; r < cols + J; ++r)
            for (int k = 0; k < J; ++k) res[k] += rhs[(size_t)r * J + k] * rhs[(size_t)r * J + k];
        for (double& v : res) v = std::sqrt(v);
    }
    // back substitution for the cols x J coefficients, column by column of the
    // triangle (the right-hand side rows above are updated as each row is solved)
    void solve(std::vector<double>& Y) {
        double dmax = 0.0;
        for (int c = 0; c < cols; ++c) dmax = std::max(dmax, std::fabs(w(c, c)));
        Y.assign((size_t)cols * J, 0.0);
        std::vector<double> t(rhs.begin(), rhs.begin() + (size_t)cols * J);
        for (int c = cols - 1; c >= 0; --c) {
            const double d = w(c, c);
            if (dead[c] || !(std::fabs(d) > 1e-13 * dmax)) continue;
            double* y = &Y[(size_t)c * J];
            for (int k = 0; k < J; ++k) y[k] = t[(size_t)c * J + k] / d;
            for (int r = 0; r < c; ++r) {
                const double a = w(r, c);
                if (a == 0.0) continue;
                double* tr = &t[(size_t)r * J];
                for (int k = 0; k < J; ++k) tr[k] -= a * y[k];
            }
        }
    }
};

template <typename T>
mhd_status block_gram(DevShared& S, const T* A, const T* B, int J, hipStream_t st, std::vector<double>& G) {
    GmresWork& W = S.gw;
    const int64_t n = S.mesh->n;
    const int64_t J2 = (int64_t)J * J;
    const int nb = (int)std::max<int64_t>(16, std::min<int64_t>(256, (W.partial_len - 1024) / J2));
    switch (J) {
        case 16: hipLaunchKernelGGL((k_bgram<T, 1>), dim3(nb), dim3(kBlock), 0, st, A, B, n, W.partial); break;
        case 32: hipLaunchKernelGGL((k_bgram<T, 2>), dim3(nb), dim3(kBlock), 0, st, A, B, n, W.partial); break;
        case 64: hipLaunchKernelGGL((k_bgram<T, 4>), dim3(nb), dim3(kBlock), 0, st, A, B, n, W.partial); break;
        default: hipLaunchKernelGGL((k_bgram<T, 8>), dim3(nb), dim3(kBlock), 0, st, A, B, n, W.partial); break;
    }
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(J2)), dim3(kBlock), 0, st, (const double*)W.partial, nb, J2, W.bmat,
                       0);
    LAUNCH_CHECK();
    G.resize(J2);
    MHD_HIP(hipMemcpyAsync(G.data(), W.bmat, sizeof(double) * J2, hipMemcpyDeviceToHost, st));
    MHD_HIP(hipStreamSynchronize(st));
    return MHD_OK;
}

template <typename T, int MODE>
mhd_status block_mm(DevShared& S, const T* A, const std::vector<double>& M, T* C, int J, hipStream_t st) {
    GmresWork& W = S.gw;
    double* dM = W.bmat + (size_t)J * J;   // the Gram result occupies the first J^2 entries
    MHD_HIP(hipMemcpyAsync(dM, M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice, st));
    const int64_t n = S.mesh->n;
    const int rpb = kBlock / J;
    const unsigned grid = (unsigned)std::min<int64_t>(4096, (n + rpb - 1) / rpb);
    hipLaunchKernelGGL((k_bmm<T, MODE>), dim3(grid), dim3(kBlock), sizeof(double) * J * J, st, A, (const double*)dM,
                       C, n, J);
    LAUNCH_CHECK();
    // M lives in host memory the next call may overwrite: wait for the copy
    MHD_HIP(hipStreamSynchronize(st));
    return MHD_OK;
}

// Block GMRES inside FP64 iterative refinement (adaptive mode): each cycle
// orthonormalises R = b - S x (deflating dependent columns), runs `restart`
// block Arnoldi steps with the right preconditioner, solves the block least
// squares problem on the host and adds the correction.
template <typename T>
mhd_status block_gmres_solve(DevShared& S, const double* b, double* x, int J, const mhd_solver_opts& o,
                             mhd_solve_stats* stt, hipStream_t st) {
    DevMesh& m = *S.mesh;
    GmresWork& G = S.gw;
    if (!(J == 16 || J == 32 || J == 64 || J == 128) || !G.bmat) {
        set_error("block GMRES needs J in {16, 32, 64, 128} and a handle with J_max <= 128");
        return MHD_EINVAL;
    }
    const int64_t n = m.n;
    const int mres = std::max(1, std::min(o.restart > 0 ? o.restart : G.restart, G.restart));
    const int sweeps = std::max(1, o.jacobi_sweeps);
    const double omega = o.jacobi_omega > 0 ? o.jacobi_omega : kJacobiOmega;
    // deflation: a pivot below 1e-5 (FP32 basis) or 1e-7 (FP64) of the largest, the
    // rounding level of a Cholesky update of the Gram matrix
    const double tol2 = sizeof(T) == 4 ? 1e-10 : 1e-14;
    const int check = std::max(1, o.check_every);
    Ops<T> ops(S, J, st);
    ops.fused_mg = o.mg_unfused == 0;
    ops.mg_cycles = o.mg_cycles == 2 ? 2 : 1;
    ops.mg_post = o.mg_post;
    BlockQR qr;
    qr.J = J;
    const bool keepz = sizeof(T) == 4 && G.zbasis != nullptr;
    const size_t zblk = (((size_t)n * S.Jmax * sizeof(float)) + 255) & ~(size_t)255;
    auto zslot = [&](int k) { return (T*)((char*)G.zbasis + (size_t)k * zblk); };
    double* hbeta = G.host_res + J;
    double* hbn = G.host_res + 2 * J;
    mhd_status rc;
    if ((rc = ops.colnorm(b, G.bnorm))) return rc;
    if ((rc = sync_copy(hbn, G.bnorm, J, st))) return rc;
    int iters = 0, cycles = 0, rank_min = J;
    double maxrel = 0.0;
    bool conv = false;
    std::vector<int> first_met(J, -1);
    std::vector<double> Gm, Minv, Cm, C0, Y;
    BlockLSQ lsq;   // host least squares, storage reused across the cycles
    while (true) {
        if ((rc = saddle_residual64(S, b, x, G.r64, J, st))) return rc;
        if ((rc = ops.colnorm(G.r64, G.beta))) return rc;
        if ((rc = sync_copy(hbeta, G.beta, J, st))) return rc;
        maxrel = 0.0;
        bool bad = false;
        for (int j = 0; j < J; ++j) {
            const double rel = hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j];
            if (!std::isfinite(rel)) bad = true;
            maxrel = std::max(maxrel, rel);
            if (first_met[j] < 0 && rel <= o.rtol) first_met[j] = iters;
        }
        if (bad) {
            set_error("mhd_ens_solve: non-finite residual");
            return MHD_ENOCONV;
        }
        if (maxrel <= o.rtol) {
            conv = true;
            break;
        }
        if (iters >= o.maxit) break;
        // R in the inner precision, orthonormalised: R = V0 C0
        T* R = (T*)G.wbuf;
        hipLaunchKernelGGL((k_convert<T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, (const double*)G.r64, R, n * J);
        LAUNCH_CHECK();
        T* V0 = basis_ptr<T>(S, 0);
        if ((rc = block_gram<T>(S, R, R, J, st, Gm))) return rc;
        int p = qr.factor(Gm, tol2, Minv, C0);
        if ((rc = block_mm<T, 0>(S, R, Minv, V0, J, st))) return rc;
        if ((rc = block_gram<T>(S, V0, V0, J, st, Gm))) return rc;   // second pass
        qr.factor(Gm, tol2, Minv, Cm);
        if ((rc = block_mm<T, 0>(S, V0, Minv, R, J, st))) return rc;
        MHD_HIP(hipMemcpyAsync(V0, R, sizeof(T) * (size_t)n * J, hipMemcpyDeviceToDevice, st));
        {
            std::vector<double> t((size_t)J * J, 0.0);   // Cm C0, rows of C0 streamed
            for (int i = 0; i < J; ++i) {
                double* tr = &t[(size_t)i * J];
                for (int q = 0; q < J; ++q) {
                    const double a = Cm[(size_t)i * J + q];
                    if (a == 0.0) continue;
                    const double* cr = &C0[(size_t)q * J];
                    for (int k = 0; k < J; ++k) tr[k] += a * cr[k];
                }
            }
            C0.swap(t);
        }
        rank_min = std::min(rank_min, p);
        // block Arnoldi
        // H[i * mres + k]: block (i, k), J x J, sized when block column k is formed
        std::vector<std::vector<double>> H((size_t)(mres + 1) * mres);
        int kd = 0;
        lsq.reset(J, mres, C0);
        std::vector<double> lsres;
        for (int k = 0; k < mres && iters < o.maxit; ++k) {
            T* vk = basis_ptr<T>(S, k);
            T* z = keepz ? zslot(k) : (T*)G.zbuf;
            T* w = basis_ptr<T>(S, k + 1);
            if ((rc = ops.precond(vk, z, sweeps, omega))) return rc;
            if ((rc = ops.saddle(z, w))) return rc;
            for (int i = 0; i <= k + 1; ++i) H[(size_t)i * mres + k].assign((size_t)J * J, 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<std::vector<double>> hk(k + 1);
                for (int i = 0; i <= k; ++i)
                    if ((rc = block_gram<T>(S, basis_ptr<T>(S, i), w, J, st, hk[i]))) return rc;
                for (int i = 0; i <= k; ++i) {
                    if ((rc = block_mm<T, 1>(S, basis_ptr<T>(S, i), hk[i], w, J, st))) return rc;
                    for (size_t q = 0; q < hk[i].size(); ++q) H[(size_t)i * mres + k][q] += hk[i][q];
                }
            }
            if ((rc = block_gram<T>(S, w, w, J, st, Gm))) return rc;
            const int pk = qr.factor(Gm, tol2, Minv, Cm);
            T* tmp = (T*)G.wbuf;
            if ((rc = block_mm<T, 0>(S, w, Minv, tmp, J, st))) return rc;
            if ((rc = block_gram<T>(S, tmp, tmp, J, st, Gm))) return rc;
            std::vector<double> Minv2, C2;
            qr.factor(Gm, tol2, Minv2, C2);
            if ((rc = block_mm<T, 0>(S, tmp, Minv2, w, J, st))) return rc;
            std::vector<double>& Hn = H[(size_t)(k + 1) * mres + k];   // C2 Cm, rows of Cm streamed
            for (int i = 0; i < J; ++i) {
                double* hr = &Hn[(size_t)i * J];
                for (int q = 0; q < J; ++q) {
                    const double a = C2[(size_t)i * J + q];
                    if (a == 0.0) continue;
                    const double* cr = &Cm[(size_t)q * J];
                    for (int c = 0; c < J; ++c) hr[c] += a * cr[c];
                }
            }
            rank_min = std::min(rank_min, pk);
            ++iters;
            kd = k + 1;
            lsq.add_block(k, H);
            if (pk == 0) break;   // the block Krylov space is exhausted
            if (kd % check == 0 && kd < mres) {   // the members' least-squares residuals so far
                lsq.residuals(lsres);
                bool done = true;
                for (int j = 0; j < J; ++j)
                    if (!(lsres[j] <= std::max(o.inner_rtol * hbeta[j], 0.5 * o.rtol * hbn[j]))) done = false;
                if (done) break;
            }
        }
        // block least squares and the correction d = P^-1 (V Y) (or Z Y with Z kept)
        lsq.solve(Y);
        T* u = (T*)G.wbuf;
        for (int k = 0; k < kd; ++k) {
            std::vector<double> Yk(Y.begin() + (size_t)k * J * J, Y.begin() + (size_t)(k + 1) * J * J);
            const T* src = keepz ? zslot(k) : basis_ptr<T>(S, k);
            if (k == 0) {
                if ((rc = block_mm<T, 0>(S, src, Yk, u, J, st))) return rc;
            } else if ((rc = block_mm<T, 2>(S, src, Yk, u, J, st))) {
                return rc;
            }
        }
        const T* d = u;
        if (!keepz) {
            if ((rc = ops.precond(u, (T*)G.zbuf, sweeps, omega))) return rc;
            d = (const T*)G.zbuf;
        }
        if (kd > 0) {
            hipLaunchKernelGGL((k_add_to64<T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, x, d, n * J);
            LAUNCH_CHECK();
        }
        ++cycles;
        if (kd == 0) break;
    }
    if (stt) {
        stt->iters = iters;
        stt->cycles = cycles;
        stt->max_relres = maxrel;
        stt->converged = conv ? 1 : 0;
        stt->nonfinite = 0;
        stt->min_block_rank = rank_min;
        stt->norm_clamps = 0;
        stt->compacted = 0;
        for (int j = 0; j < J; ++j) {
            if (stt->relres) stt->relres[j] = hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j];
            if (stt->member_iters) stt->member_iters[j] = first_met[j] < 0 ? iters : first_met[j];
        }
    }
    if (!conv) {
        set_error("mhd_ens_solve: maxit reached before rtol (best iterate written)");
        return MHD_ENOCONV;
    }
    return MHD_OK;
}

}  // namespace

// ------------------------------------------------------------------ allocation and entry
mhd_status alloc_gmres(DevShared& S, int restart, bool compact) {
    DevMesh& m = *S.mesh;
    GmresWork& G = S.gw;
    G.restart = restart;
    G.nrows = m.n;
    G.Jmax = S.Jmax;
    const size_t blk = slot_bytes(m.n, S.Jmax);
    auto A = [&](void** p, size_t bytes) -> mhd_status {
        hipError_t e = dev_malloc(p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
            return MHD_ENOMEM;
        }
        S.allocs.push_back(*p);
        return MHD_OK;
    };
    mhd_status rc;
    if ((rc = A(&G.basis, blk * (restart + 1)))) return rc;
    if ((rc = A(&G.zbuf, blk))) return rc;
    if ((rc = A(&G.wbuf, blk))) return rc;
    if ((rc = A(&G.tbuf, blk))) return rc;
    if ((rc = A(&G.z2buf, blk))) return rc;
    if ((rc = A((void**)&G.r64, blk))) return rc;
    const size_t J8 = (size_t)S.Jmax * sizeof(double);
    if ((rc = A((void**)&G.H, J8 * (restart + 1) * restart))) return rc;
    if ((rc = A((void**)&G.cs, J8 * restart))) return rc;
    if ((rc = A((void**)&G.sn, J8 * restart))) return rc;
    if ((rc = A((void**)&G.g, J8 * (restart + 1)))) return rc;
    if ((rc = A((void**)&G.y, J8 * restart))) return rc;
    if ((rc = A((void**)&G.beta, J8))) return rc;
    if ((rc = A((void**)&G.bnorm, J8))) return rc;
    if ((rc = A((void**)&G.hcol, J8 * 2 * (kMaxRestart + 1)))) return rc;
    if ((rc = A((void**)&G.res, J8 * 3))) return rc;   // estimates, new-vector norms, norm-clamp counts
    if (compact) {
        if ((rc = A((void**)&G.cb, (size_t)m.n * J8))) return rc;
        if ((rc = A((void**)&G.cx, (size_t)m.n * J8))) return rc;
        if ((rc = A((void**)&G.cidx, sizeof(int32_t) * (size_t)S.Jmax))) return rc;
    }
    if (S.Jmax <= kBlockMaxJ && (rc = A((void**)&G.bmat, sizeof(double) * 2 * (size_t)S.Jmax * S.Jmax))) return rc;
    G.nblk_cap = std::min(kRedBlocks, std::max(64, 524288 / S.Jmax));
    G.partial_len = (int64_t)G.nblk_cap * (restart + 2) * S.Jmax + 1024;
    if ((rc = A((void**)&G.partial, sizeof(double) * G.partial_len))) return rc;
    if ((rc = A((void**)&G.dptrs, sizeof(void*) * (kMaxRestart + 2)))) return rc;
    std::vector<void*> ptrs(restart + 1);
    for (int i = 0; i <= restart; ++i) ptrs[i] = (char*)G.basis + (size_t)i * blk;
    MHD_HIP(hipMemcpy(G.dptrs, ptrs.data(), sizeof(void*) * (restart + 1), hipMemcpyHostToDevice));
    // FP32 solves keep M^-1 v_k of every inner iteration (slots of n x Jmax floats)
    const size_t zblk = (((size_t)m.n * S.Jmax * sizeof(float)) + 255) & ~(size_t)255;
    if ((rc = A(&G.zbasis, zblk * restart))) return rc;
    if ((rc = A((void**)&G.zptrs, sizeof(void*) * (kMaxRestart + 1)))) return rc;
    std::vector<void*> zp(restart);
    for (int i = 0; i < restart; ++i) zp[i] = (char*)G.zbasis + (size_t)i * zblk;
    MHD_HIP(hipMemcpy(G.zptrs, zp.data(), sizeof(void*) * restart, hipMemcpyHostToDevice));
    if ((rc = A(&G.dense_part, (size_t)kDenseKS * m.levels.back().n * S.Jmax * sizeof(double)))) return rc;
    for (size_t l = 0; l < m.levels.size(); ++l) {
        size_t lb = (size_t)m.levels[l].n * S.Jmax * sizeof(double);
        void *a, *b, *c, *d;
        if ((rc = A(&a, lb))) return rc;
        if ((rc = A(&b, lb))) return rc;
        if ((rc = A(&c, lb))) return rc;
        if ((rc = A(&d, lb))) return rc;
        G.mg_x.push_back(a);
        G.mg_x2.push_back(b);
        G.mg_b.push_back(c);
        G.mg_r.push_back(d);
    }
    if ((rc = A(&G.mg_y0, (size_t)m.levels[0].n * S.Jmax * sizeof(double)))) return rc;
    hipError_t e = hipHostMalloc((void**)&G.host_res, sizeof(double) * 3 * S.Jmax, hipHostMallocDefault);
    if (e != hipSuccess) {
        set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
        return MHD_ENOMEM;
    }
    return MHD_OK;
}

// No tuning and no allocation here: the node-row operators run the plans in the
// process-wide table (filled by mhd_ens_prepare / mhd_ens_autotune / context
// creation) where this handle holds their data, and the default plans otherwise.
mhd_status solve_shared(DevShared& S, const double* rhs, double* x, int J, const mhd_solver_opts& o,
                        mhd_solve_stats* st, hipStream_t s) {
    if (o.block_krylov) {
        if (o.precision == MHD_FP32_IR) return block_gmres_solve<float>(S, rhs, x, J, o, st, s);
        return block_gmres_solve<double>(S, rhs, x, J, o, st, s);
    }
    if (o.precision == MHD_FP32_IR) return gmres_solve<float>(S, rhs, x, J, o, st, s);
    return gmres_solve<double>(S, rhs, x, J, o, st, s);
}

// Final FP64 residuals of a solve: rel_j = ||b_j - S x_j|| / ||b_j|| per member
// into st (max_relres, nonfinite, relres[] if given).  Synchronises st.
mhd_status residual_report(DevShared& S, const double* b, const double* x, int J, mhd_solve_stats* out,
                           hipStream_t st) {
    GmresWork& G = S.gw;
    Ops<double> ops(S, J, st);
    mhd_status rc;
    if ((rc = saddle_residual64(S, b, x, G.r64, J, st))) return rc;
    if ((rc = ops.colnorm(G.r64, G.beta))) return rc;
    if ((rc = ops.colnorm(b, G.bnorm))) return rc;
    double* hbeta = G.host_res + J;
    double* hbn = G.host_res + 2 * J;
    if ((rc = sync_copy(hbeta, G.beta, J, st))) return rc;
    if ((rc = sync_copy(hbn, G.bnorm, J, st))) return rc;
    double mx = 0.0;
    int bad = 0;
    for (int j = 0; j < J; ++j) {
        const double rel = hbn[j] > 0 ? hbeta[j] / hbn[j] : hbeta[j];
        if (!std::isfinite(rel)) ++bad;
        else mx = std::max(mx, rel);
        if (out->relres) out->relres[j] = rel;
    }
    out->max_relres = bad ? NAN : mx;
    out->nonfinite = bad;
    out->norm_clamps = norm_clamp_count(G, J, st);
    return MHD_OK;
}

mhd_status saddle_residual64(DevShared& S, const double* b, const double* x, double* r, int J, hipStream_t st) {
    const bool aligned = (((uintptr_t)b | (uintptr_t)x | (uintptr_t)r) % 16) == 0;
    const NodePlan p = align_plan(get_plan(*S.mesh, J, 8, MHD_TUNE_RESIDUAL), aligned);
    return launch_saddle_plan<double, 1>(p, S, x, b, r, J, st);
}

hipError_t launch_reduce_rows(const double* partial, int nblk, int64_t width, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(width)), dim3(kBlock), 0, s, partial, nblk, width, out, 0);
    return hipGetLastError();
}

mhd_status spmm_shared(DevShared& S, const void* x, void* y, int J, int precision, hipStream_t st) {
    if (precision == MHD_FP32_IR) {
        Ops<float> ops(S, J, st);
        return ops.saddle((const float*)x, (float*)y);
    }
    Ops<double> ops(S, J, st);
    return ops.saddle((const double*)x, (double*)y);
}

mhd_status timer_enable(int on) {
    if (on) {
        if (g_timer.pool.empty()) {
            g_timer.pool.resize(8192);
            for (auto& e : g_timer.pool) MHD_HIP(hipEventCreate(&e));
        }
        g_timer.used = 0;
    } else {
        hipError_t e = timer_fold();
        if (e != hipSuccess) {
            set_error(std::string("timer: ") + hipGetErrorString(e));
            return MHD_EHIP;
        }
    }
    if (on) {
        g_timer.ms = 0.0;
        g_timer.launches = 0;
        g_timer.nJ32 = g_timer.nJ64 = 0.0;
    }
    g_timer.on = on != 0;
    return MHD_OK;
}

mhd_status timer_op(int op) {
    if (op != MHD_TUNE_SADDLE && op != MHD_TUNE_JACOBI) {
        set_error("mhd_ens_timer_op: op must be MHD_TUNE_SADDLE or MHD_TUNE_JACOBI");
        return MHD_EINVAL;
    }
    g_timer.op = op;
    return MHD_OK;
}

mhd_status timer_read(double* ms, int64_t* launches, double* nJ32, double* nJ64) {
    hipError_t e = timer_fold();
    if (e != hipSuccess) {
        set_error(std::string("timer: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    if (ms) *ms = g_timer.ms;
    if (launches) *launches = g_timer.launches;
    if (nJ32) *nJ32 = g_timer.nJ32;
    if (nJ64) *nJ64 = g_timer.nJ64;
    return MHD_OK;
}

hipError_t launch_pressure_zero_mean(const DevMesh& m, double* p, int J, double* partial, hipStream_t st) {
    RedShape rs = cap_blocks(red_shape(m.nP1, J, 1), std::min(kRedBlocks, std::max(64, 524288 / J)));
    hipLaunchKernelGGL(k_wsum, rs.grid, dim3(kBlock), 0, st, (const double*)p, (const double*)m.mp, (int64_t)m.nP1, J,
                       rs.CW, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* sums = partial + (int64_t)rs.nblk * J;
    hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(J)), dim3(kBlock), 0, st, (const double*)partial, rs.nblk, (int64_t)J,
                       sums, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double area = 0.0;
    for (double v : m.host.mp) area += v;
    hipLaunchKernelGGL(k_sub_mean, dim3(ew_grid((int64_t)m.nP1 * J)), dim3(kBlock), 0, st, p, (const double*)sums,
                       1.0 / area, (int64_t)m.nP1, J);
    return hipGetLastError();
}

}  // namespace mhd
