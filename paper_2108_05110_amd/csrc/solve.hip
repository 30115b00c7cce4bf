// Batched solver of libmhd_ens (gfx950): S X = B with one shared saddle-point
// matrix S = [[A (x) I_2, B^T], [B, D_p]] and J member columns (paper,
// Section 1: A [x_1|...|x_J] = [b_1|...|b_J]; Section 4: two Oseen-type
// problems per step).
//
// Method: right-preconditioned restarted GMRES with one Arnoldi process per
// member (per-member Hessenberg matrices and Givens rotations in FP64), one
// SpMM over all J columns per iteration.  Preconditioner (block upper
// triangular): z_p = S_hat^{-1} r_p with the Cahouet-Chabard approximation
// S_hat^{-1} = -(1/dt) L_p^{-1} - nu_c M_p^{-1} (L_p: P1 Laplacian, one
// geometric multigrid V-cycle with damped Jacobi smoothing; M_p lumped P1
// mass), then z_u = damped Jacobi sweeps on A for r_u - B^T z_p.  The outer
// loop is FP64 iterative refinement: r = b - S x in FP64, a GMRES cycle in
// the inner precision (FP32 or FP64) on r, x += d.
//
// Every kernel streams member blocks row-major (member index fastest); rows
// are spread over the 8 XCDs in contiguous ranges.  Column reductions go
// through per-block partials and a fixed-order second pass (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

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
// MODE 3: y = x + w dinv (b - A x) ; MODE 4: y = w dinv b (x unused)
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
        if (MODE != 4)
            for (int32_t p = p0; p < p1; ++p) s += val[p] * x[(int64_t)col[p] * J + j];
        const int64_t o = r * J + j;
        if (MODE == 0) y[o] = s;
        if (MODE == 1) y[o] += s;
        if (MODE == 2) y[o] = b[o] - s;
        if (MODE == 3) y[o] = x[o] + omega * dinv[r] * (b[o] - s);
        if (MODE == 4) y[o] = omega * dinv[r] * b[o];
    }
}

// x = Cinv b on the coarsest level (dense, n <= a few hundred): one block per
// row and member tile; the 4 wavefronts split the columns, fixed-order sum in LDS
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense(const T* __restrict__ C, const T* __restrict__ b, T* __restrict__ x,
                                                  int n, int J) {
    __shared__ T red[kBlock];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.x;
    const int j = blockIdx.y * 64 + lane;
    T s = 0;
    if (j < J)
        for (int c = wave; c < n; c += kBlock / 64) s += C[(int64_t)r * n + c] * b[(int64_t)c * J + j];
    red[threadIdx.x] = s;
    __syncthreads();
    if (wave == 0 && j < J) x[(int64_t)r * J + j] = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
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

// partial[((c0 + i) * J + j) * nblk + block] = sum over rows of V_i[r, j] * w[r, j], i < nb
template <typename T, int VEC, int NB>
__global__ void __launch_bounds__(kBlock) k_dots(const T* const* __restrict__ V, int c0, int nb, const T* __restrict__ w,
                                                 int64_t n, int J, int CW, double* __restrict__ partial) {
    __shared__ double red[kBlock];
    const ColMap c = colmap(CW, VEC, J);
    double acc[NB][VEC];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int u = 0; u < VEC; ++u) acc[i][u] = 0.0;
    if (c.ok) {
        const T* vp[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) vp[i] = (i < nb) ? V[c0 + i] : nullptr;
        for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG) {
            T wv[VEC];
            vload<T, VEC>(wv, w + r * J + c.jb);
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i < nb) {
                    T vv[VEC];
                    vload<T, VEC>(vv, vp[i] + r * J + c.jb);
#pragma unroll
                    for (int u = 0; u < VEC; ++u) acc[i][u] += (double)vv[u] * (double)wv[u];
                }
        }
    }
    const int64_t nblk = gridDim.x;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (i < nb) {
#pragma unroll
            for (int u = 0; u < VEC; ++u) {
                double sv = block_colsum(acc[i][u], c, red, CW);
                if (c.ty == 0 && c.ok) partial[((int64_t)(c0 + i) * J + c.jb + u) * nblk + blockIdx.x] = sv;
            }
        }
    }
}

// w -= sum_{i<nb} h[i*J + j] V_i ; partial[j * nblk + block] = sum over rows of w^2
template <typename T, int VEC>
__global__ void __launch_bounds__(kBlock) k_update(const T* const* __restrict__ V, int nb, const double* __restrict__ h,
                                                   T* __restrict__ w, int64_t n, int J, int CW,
                                                   double* __restrict__ partial) {
    __shared__ double red[kBlock];
    const ColMap c = colmap(CW, VEC, J);
    double acc[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
    if (c.ok) {
        for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG) {
            T wv[VEC];
            vload<T, VEC>(wv, w + r * J + c.jb);
            for (int i = 0; i < nb; ++i) {
                T vv[VEC];
                vload<T, VEC>(vv, V[i] + r * J + c.jb);
#pragma unroll
                for (int u = 0; u < VEC; ++u) wv[u] -= (T)h[(int64_t)i * J + c.jb + u] * vv[u];
            }
            vstore<T, VEC>(w + r * J + c.jb, wv);
#pragma unroll
            for (int u = 0; u < VEC; ++u) acc[u] += (double)wv[u] * (double)wv[u];
        }
    }
    const int64_t nblk = gridDim.x;
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
        double sv = block_colsum(acc[u], c, red, CW);
        if (c.ty == 0 && c.ok) partial[((int64_t)c.jb + u) * nblk + blockIdx.x] = sv;
    }
}

// partial[j * nblk + block] = sum over rows of a[r, j]^2 (FP64 blocks)
template <int VEC>
__global__ void __launch_bounds__(kBlock) k_colsq(const double* __restrict__ a, int64_t n, int J, int CW,
                                                  double* __restrict__ partial) {
    __shared__ double red[kBlock];
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
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
        double sv = block_colsum(acc[u], c, red, CW);
        if (c.ty == 0 && c.ok) partial[((int64_t)c.jb + u) * nblk + blockIdx.x] = sv;
    }
}

// u = sum_{i<nb} y[i*J + j] V_i
template <typename T, int VEC>
__global__ void __launch_bounds__(kBlock) k_combine(const T* const* __restrict__ V, int nb, const double* __restrict__ yv,
                                                    T* __restrict__ u, int64_t n, int J, int CW) {
    const ColMap c = colmap(CW, VEC, J);
    if (!c.ok) return;
    for (int64_t r = (int64_t)blockIdx.x * c.RG + c.ty; r < n; r += (int64_t)gridDim.x * c.RG) {
        T s[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) s[q] = 0;
        for (int i = 0; i < nb; ++i) {
            T vv[VEC];
            vload<T, VEC>(vv, V[i] + r * J + c.jb);
#pragma unroll
            for (int q = 0; q < VEC; ++q) s[q] += (T)yv[(int64_t)i * J + c.jb + q] * vv[q];
        }
        vstore<T, VEC>(u + r * J + c.jb, s);
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

// Givens step k for every member (FP64): rotate column k of H, new rotation, update g.
__global__ void k_givens(double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                         double* __restrict__ g, const double* __restrict__ hcol, const double* __restrict__ hn,
                         double* __restrict__ res, int k, int m, int J) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    double h[kMaxRestart + 1];
    for (int i = 0; i <= k; ++i) h[i] = hcol[i * J + j];
    h[k + 1] = hn[j];
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

// record the start (before = true) or the end of one timed launch on stream st
void timer_mark(hipStream_t st, bool before) {
    if (!g_timer.on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    if (before && g_timer.used + 2 > g_timer.pool.size()) (void)timer_fold();
    if (g_timer.used < g_timer.pool.size()) (void)hipEventRecord(g_timer.pool[g_timer.used++], st);
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

// ------------------------------------------------------------------ host-side operators
template <typename T>
struct Ops {
    DevShared& S;
    int J;
    hipStream_t st;
    int JP;

    Ops(DevShared& s, int j, hipStream_t stream) : S(s), J(j), st(stream), JP(pick_jp(j)) {}

    mhd_status saddle(const T* x, T* y) {
        DevMesh& m = *S.mesh;
        int64_t units = (int64_t)m.nP2 + m.nP1;
        timer_mark(st, true);
        mhd_status rc = MHD_OK;
        const bool aligned = (((uintptr_t)x | (uintptr_t)y) % 16) == 0;
        const int fv = fast_vec(J, aligned ? (sizeof(T) == 4 ? 4 : 2) : 1);
        if (fv) {
            rc = with_vec<T>(fv, [&](auto V) -> mhd_status {
                hipLaunchKernelGGL((k_saddle_v<T, decltype(V)::value, 0>), node_grid(units, J, fv), dim3(kBlock), 0,
                                   st, m.A_rowptr, m.A_col, Vals<T>::A(S), m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S),
                                   m.B_rowptr, m.B_col, Vals<T>::B(S), Vals<T>::dp(m), x, (const T*)nullptr, y, m.nP2,
                                   m.nP1, J);
                LAUNCH_CHECK();
                return MHD_OK;
            });
        } else {
            hipLaunchKernelGGL((k_saddle<T, 0>), dim3(grid_for(units, JP)), dim3(kBlock), 0, st, m.A_rowptr, m.A_col,
                               Vals<T>::A(S), m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S), m.B_rowptr, m.B_col,
                               Vals<T>::B(S), Vals<T>::dp(m), x, (const T*)nullptr, y, m.nP2, m.nP1, J, JP);
            LAUNCH_CHECK();
        }
        if (rc) return rc;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (g_timer.on && hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            timer_mark(st, false);
            g_timer.launches++;
            (sizeof(T) == 4 ? g_timer.nJ32 : g_timer.nJ64) += (double)J;
        }
        return MHD_OK;
    }

    template <int MODE>
    mhd_status csr(const DevCSR<double>& c, const T* dinv, const T* x, const T* b, T* y, T omega) {
        hipLaunchKernelGGL((k_csr<T, MODE>), dim3(grid_for(c.nrows, JP)), dim3(kBlock), 0, st, c.rowptr, c.col,
                           Vals<T>::csr(c), dinv, x, b, y, c.nrows, J, JP, omega);
        LAUNCH_CHECK();
        return MHD_OK;
    }

    // One V(2,2)-cycle with damped Jacobi smoothing on level l for L_l x = b.
    // Uses the level's buffers x, x2, r and the next level's b and x.  Returns
    // the buffer holding the result in *out.
    mhd_status vcycle(int l, const T* b, T** out) {
        DevMesh& m = *S.mesh;
        const DevLevel& Lv = m.levels[l];
        T* x = (T*)S.gw.mg_x[l];
        mhd_status rc;
        if (l + 1 == (int)m.levels.size()) {
            hipLaunchKernelGGL((k_dense<T>), dim3(Lv.n, (J + 63) / 64), dim3(kBlock), 0, st, Vals<T>::cinv(Lv), b, x,
                               Lv.n, J);
            LAUNCH_CHECK();
            *out = x;
            return MHD_OK;
        }
        const T omega = (T)0.8;
        T* x2 = (T*)S.gw.mg_x2[l];
        T* r = (T*)S.gw.mg_r[l];
        T* bc = (T*)S.gw.mg_b[l + 1];
        const T* dinv = Vals<T>::dinv(Lv);
        if ((rc = csr<4>(Lv.L, dinv, nullptr, b, x, omega))) return rc;   // x  = w D^-1 b
        if ((rc = csr<3>(Lv.L, dinv, x, b, x2, omega))) return rc;        // x2 = x + w D^-1 (b - L x)
        if ((rc = csr<2>(Lv.L, dinv, x2, b, r, omega))) return rc;        // r  = b - L x2
        if ((rc = csr<0>(Lv.R, dinv, r, nullptr, bc, omega))) return rc;  // bc = R r
        T* xc = nullptr;
        if ((rc = vcycle(l + 1, bc, &xc))) return rc;
        if ((rc = csr<1>(Lv.P, dinv, xc, nullptr, x2, omega))) return rc; // x2 += P xc
        if ((rc = csr<3>(Lv.L, dinv, x2, b, x, omega))) return rc;        // post-smoothing
        if ((rc = csr<3>(Lv.L, dinv, x, b, x2, omega))) return rc;
        *out = x2;
        return MHD_OK;
    }

    // z = P^{-1} v (block upper-triangular preconditioner)
    mhd_status precond(const T* v, T* z, int sweeps) {
        DevMesh& m = *S.mesh;
        const int64_t off = 2 * (int64_t)m.nP2 * J;
        const T* vp = v + off;
        T* zp = z + off;
        mhd_status rc;
        T* xmg = nullptr;
        if ((rc = vcycle(0, vp, &xmg))) return rc;
        hipLaunchKernelGGL((k_schur<T>), dim3(grid_for(m.nP1, JP)), dim3(kBlock), 0, st, xmg, vp, m.pin, zp, m.nP1,
                           J, JP);
        LAUNCH_CHECK();
        const T omega = (T)0.7;
        T* t = (T*)S.gw.tbuf;
        T* za = z;
        T* zb = (T*)S.gw.z2buf;
        const int fv = fast_vec(J, sizeof(T) == 4 ? 4 : 2);
        if (fv) {
            rc = with_vec<T>(fv, [&](auto V) -> mhd_status {
                constexpr int VV = decltype(V)::value;
                hipLaunchKernelGGL((k_velo_v<T, VV, true>), node_grid(m.nP2, J, fv), dim3(kBlock), 0, st,
                                   m.Bt_rowptr, m.Bt_col, Vals<T>::Bt(S), Vals<T>::dA(S), v, (const T*)zp, t,
                                   (const T*)nullptr, za, m.nP2, J, omega);
                LAUNCH_CHECK();
                for (int s = 1; s < sweeps; ++s) {
                    hipLaunchKernelGGL((k_velo_v<T, VV, false>), node_grid(m.nP2, J, fv), dim3(kBlock), 0, st,
                                       m.A_rowptr, m.A_col, Vals<T>::A(S), Vals<T>::dA(S), (const T*)nullptr,
                                       (const T*)nullptr, t, (const T*)za, zb, m.nP2, J, omega);
                    LAUNCH_CHECK();
                    std::swap(za, zb);
                }
                return MHD_OK;
            });
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL((k_velo_first<T>), dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, st, m.Bt_rowptr,
                               m.Bt_col, Vals<T>::Bt(S), Vals<T>::dA(S), v, zp, t, za, m.nP2, J, JP, omega);
            LAUNCH_CHECK();
            for (int s = 1; s < sweeps; ++s) {
                hipLaunchKernelGGL((k_velo_sweep<T>), dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, st, m.A_rowptr,
                                   m.A_col, Vals<T>::A(S), Vals<T>::dA(S), t, za, zb, m.nP2, J, JP, omega);
                LAUNCH_CHECK();
                std::swap(za, zb);
            }
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

template <typename T>
mhd_status gmres_solve(DevShared& S, const double* b, double* x, int J, const mhd_solver_opts& o,
                       mhd_solve_stats* stt, hipStream_t st) {
    DevMesh& m = *S.mesh;
    GmresWork& G = S.gw;
    const int64_t n = m.n;
    const int mres = std::max(1, std::min(o.restart > 0 ? o.restart : G.restart, G.restart));
    const int check = std::max(1, o.check_every);
    const int sweeps = std::max(1, o.jacobi_sweeps);
    Ops<T> ops(S, J, st);
    RedShape rs = cap_blocks(red_shape(n, J, 16 / (int)sizeof(T)), G.nblk_cap);
    const int passes = o.cgs_passes > 0 ? o.cgs_passes : (sizeof(T) == 4 ? 1 : 2);
    const T* const* Vd = (const T* const*)G.dptrs;
    double* hres = G.host_res;                 // pinned, 3 J doubles: residuals, beta, bnorm
    double* hbeta = G.host_res + J;
    double* hbn = G.host_res + 2 * J;
    double* hcol2 = G.hcol + (int64_t)(kMaxRestart + 1) * J;
    double* hn = G.res + J;
    mhd_status rc;
    // fixed schedule: fixed_cycles refinement cycles of mres inner iterations,
    // no host synchronisation (graph-capturable)
    const bool fixed = o.fixed_cycles > 0;
    if (!fixed) {
        if ((rc = ops.colnorm(b, G.bnorm))) return rc;
        if ((rc = sync_copy(hbn, G.bnorm, J, st))) return rc;
    }
    int iters = 0, cycles = 0;
    double maxrel = 0.0;
    bool conv = false;
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
        if (bad) {
            set_error("mhd_ens_solve: non-finite residual");
            if (stt) *stt = {iters, cycles, maxrel, 0};
            return MHD_ENOCONV;
        }
        if (maxrel <= o.rtol) {
            conv = true;
            break;
        }
        if (iters >= o.maxit) break;
        }
        // v0 = r / beta in the inner precision; g = beta e1
        hipLaunchKernelGGL((k_scale_cols<double, T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, (const double*)G.r64,
                           G.beta, 1, basis_ptr<T>(S, 0), n, J);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_init_g, dim3((J + 255) / 256), dim3(256), 0, st, G.g, G.beta, mres + 1, J);
        LAUNCH_CHECK();
        int kd = 0;
        for (int k = 0; k < mres && (fixed || iters < o.maxit); ++k) {
            T* vk = basis_ptr<T>(S, k);
            T* z = (T*)G.zbuf;
            T* w = basis_ptr<T>(S, k + 1);
            if ((rc = ops.precond(vk, z, sweeps))) return rc;
            if ((rc = ops.saddle(z, w))) return rc;
            // classical Gram-Schmidt (optionally with a re-orthogonalisation pass)
            for (int pass = 0; pass < passes; ++pass) {
                double* hdst = pass ? hcol2 : G.hcol;
                for (int c0 = 0; c0 <= k; c0 += 8) {
                    int nb = std::min(8, k + 1 - c0);
                    rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                        hipLaunchKernelGGL((k_dots<T, decltype(V)::value, 8>), rs.grid, dim3(kBlock), 0, st, Vd, c0, nb,
                                           (const T*)w, n, J, rs.CW, G.partial);
                        LAUNCH_CHECK();
                        return MHD_OK;
                    });
                    if (rc) return rc;
                }
                hipLaunchKernelGGL(k_reduce, dim3(reduce_grid((int64_t)(k + 1) * J)), dim3(kBlock), 0, st, G.partial,
                                   rs.nblk, (int64_t)(k + 1) * J, hdst, 0);
                LAUNCH_CHECK();
                rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
                    hipLaunchKernelGGL((k_update<T, decltype(V)::value>), rs.grid, dim3(kBlock), 0, st, Vd, k + 1,
                                       (const double*)hdst, w, n, J, rs.CW, G.partial);
                    LAUNCH_CHECK();
                    return MHD_OK;
                });
                if (rc) return rc;
            }
            hipLaunchKernelGGL(k_reduce, dim3(reduce_grid(J)), dim3(kBlock), 0, st, G.partial, rs.nblk, (int64_t)J, hn,
                               1);
            LAUNCH_CHECK();
            if (passes > 1) {
                hipLaunchKernelGGL(k_add_vec, dim3(((k + 1) * J + 255) / 256), dim3(256), 0, st, G.hcol,
                                   (const double*)hcol2, (int64_t)(k + 1) * J);
                LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_givens, dim3((J + 63) / 64), dim3(64), 0, st, G.H, G.cs, G.sn, G.g, G.hcol, hn, G.res,
                               k, mres, J);
            LAUNCH_CHECK();
            hipLaunchKernelGGL((k_scale_cols<T, T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, (const T*)w, hn, 1, w,
                               n, J);
            LAUNCH_CHECK();
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
        // x += P^{-1} (V y)
        hipLaunchKernelGGL(k_lsq, dim3((J + 63) / 64), dim3(64), 0, st, G.H, G.g, G.y, kd, mres, J);
        LAUNCH_CHECK();
        T* u = (T*)G.wbuf;
        rc = with_vec<T>(rs.VEC, [&](auto V) -> mhd_status {
            hipLaunchKernelGGL((k_combine<T, decltype(V)::value>), rs.grid, dim3(kBlock), 0, st, Vd, kd,
                               (const double*)G.y, u, n, J, rs.CW);
            LAUNCH_CHECK();
            return MHD_OK;
        });
        if (rc) return rc;
        if ((rc = ops.precond(u, (T*)G.zbuf, sweeps))) return rc;
        hipLaunchKernelGGL((k_add_to64<T>), dim3(ew_grid(n * J)), dim3(kBlock), 0, st, x, (const T*)G.zbuf, n * J);
        LAUNCH_CHECK();
        ++cycles;
    }
    if (fixed) {
        if (stt) *stt = {iters, cycles, -1.0, -1};
        return MHD_OK;
    }
    if (stt) *stt = {iters, cycles, maxrel, conv ? 1 : 0};
    if (!conv) {
        set_error("mhd_ens_solve: maxit reached before rtol (best iterate written)");
        return MHD_ENOCONV;
    }
    return MHD_OK;
}

}  // namespace

// ------------------------------------------------------------------ allocation and entry
mhd_status alloc_gmres(DevShared& S, int restart) {
    DevMesh& m = *S.mesh;
    GmresWork& G = S.gw;
    G.restart = restart;
    G.nrows = m.n;
    G.Jmax = S.Jmax;
    const size_t blk = slot_bytes(m.n, S.Jmax);
    auto A = [&](void** p, size_t bytes) -> mhd_status {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
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
    if ((rc = A((void**)&G.res, J8 * 2))) return rc;
    G.nblk_cap = std::min(kRedBlocks, std::max(64, 524288 / S.Jmax));
    G.partial_len = (int64_t)G.nblk_cap * (restart + 2) * S.Jmax + 1024;
    if ((rc = A((void**)&G.partial, sizeof(double) * G.partial_len))) return rc;
    if ((rc = A((void**)&G.dptrs, sizeof(void*) * (kMaxRestart + 2)))) return rc;
    std::vector<void*> ptrs(restart + 1);
    for (int i = 0; i <= restart; ++i) ptrs[i] = (char*)G.basis + (size_t)i * blk;
    MHD_HIP(hipMemcpy(G.dptrs, ptrs.data(), sizeof(void*) * (restart + 1), hipMemcpyHostToDevice));
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
    hipError_t e = hipHostMalloc((void**)&G.host_res, sizeof(double) * 3 * S.Jmax, hipHostMallocDefault);
    if (e != hipSuccess) {
        set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
        return MHD_ENOMEM;
    }
    return MHD_OK;
}

mhd_status solve_shared(DevShared& S, const double* rhs, double* x, int J, const mhd_solver_opts& o,
                        mhd_solve_stats* st, hipStream_t s) {
    if (o.precision == MHD_FP32_IR) return gmres_solve<float>(S, rhs, x, J, o, st, s);
    return gmres_solve<double>(S, rhs, x, J, o, st, s);
}

mhd_status saddle_residual64(DevShared& S, const double* b, const double* x, double* r, int J, hipStream_t st) {
    DevMesh& m = *S.mesh;
    const int64_t units = (int64_t)m.nP2 + m.nP1;
    const bool aligned = ((uintptr_t)b % 16 == 0) && ((uintptr_t)x % 16 == 0);
    const int fv = aligned ? fast_vec(J, 2) : (fast_vec(J, 1) ? 1 : 0);
    if (fv == 2) {
        hipLaunchKernelGGL((k_saddle_v<double, 2, 1>), node_grid(units, J, 2), dim3(kBlock), 0, st, m.A_rowptr,
                           m.A_col, Vals<double>::A(S), m.Bt_rowptr, m.Bt_col, Vals<double>::Bt(S), m.B_rowptr, m.B_col, Vals<double>::B(S), m.diagp, x, b,
                           r, m.nP2, m.nP1, J);
    } else if (fv == 1) {
        hipLaunchKernelGGL((k_saddle_v<double, 1, 1>), node_grid(units, J, 1), dim3(kBlock), 0, st, m.A_rowptr,
                           m.A_col, Vals<double>::A(S), m.Bt_rowptr, m.Bt_col, Vals<double>::Bt(S), m.B_rowptr, m.B_col, Vals<double>::B(S), m.diagp, x, b,
                           r, m.nP2, m.nP1, J);
    } else {
        int JP = pick_jp(J);
        hipLaunchKernelGGL((k_saddle<double, 1>), dim3(grid_for(units, JP)), dim3(kBlock), 0, st, m.A_rowptr, m.A_col,
                           Vals<double>::A(S), m.Bt_rowptr, m.Bt_col, Vals<double>::Bt(S), m.B_rowptr, m.B_col, Vals<double>::B(S), m.diagp, x, b, r,
                           m.nP2, m.nP1, J, JP);
    }
    LAUNCH_CHECK();
    return MHD_OK;
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
