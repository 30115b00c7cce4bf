// Adjoint kernels of libmhd_ens (gfx950): the discrete adjoint of one step of
// Algorithm 1 (paper, Section 3) for an ensemble-mean objective.
//
// With the shared matrices S_v(W^n), S_w(V^n) and the multipliers mu_v, mu_w
// from the transposed solves S^T mu = [lambda^{n+1}; 0], the adjoint state of
// time level n is
//   lambda_V_j = M mu_v/dt - c+_j K mu_v + N*(w_j') mu_v - c-_j K mu_w
//                - C(W_j)^T mu_w + mean_i C(W_i)^T mu_w - mean_i C(W_i^{n+1})^T mu_w - E_v(j)
// (and the same with v and w exchanged), where C(Z)^T mu is the transpose of
// u -> b*(u, Z, .) (the trilinear form's derivative in its convecting
// argument: fluctuation w_j' = w_j - <w> and mean <w> of the shared matrix),
// and E_v is the derivative of the eddy term through l_v^2 = max_j |v_j'|^2,
// which follows the maximising member (lowest index on ties).  Multipliers
// are taken as zero on Dirichlet rows (those rows do not depend on the state).
// Only the skew-symmetric trilinear form is differentiated.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace mhd {

namespace {

// reference-element tables of this translation unit (same contents as the
// assembly kernels' copy; each code object holds its own constant memory)
__constant__ RefTables c_ref;

}  // namespace

void upload_ref_tables_adjoint(const RefTables& t) { (void)hipMemcpyToSymbol(HIP_SYMBOL(c_ref), &t, sizeof(RefTables)); }

namespace {

constexpr int kBlock = 256;

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

struct Geo {
    double det, Ji[2][2];
};

__device__ __forceinline__ Geo load_geo(const double* geo, int64_t e) {
    Geo g;
    g.det = geo[e * 6];
    g.Ji[0][0] = geo[e * 6 + 1];
    g.Ji[0][1] = geo[e * 6 + 2];
    g.Ji[1][0] = geo[e * 6 + 3];
    g.Ji[1][1] = geo[e * 6 + 4];
    return g;
}

// masked multiplier value (zero on Dirichlet nodes)
__device__ __forceinline__ double mval(const double* mu, const uint8_t* dir, int node, int c, int J, int j) {
    return dir[node] ? 0.0 : mu[(int64_t)(2 * node + c) * J + j];
}

// C(Z)^T mu at local node a of element e, member j, both components:
// out_d = det sum_e' Ji[e'][d] sum_{x,c} Shat[x][a][c][e'] (mu_x . Z_c)
__device__ __forceinline__ void conv_adj_local(const int* t, const Geo& g, int a, const double* __restrict__ mu,
                                               const uint8_t* __restrict__ dir, const double* __restrict__ Z, int J,
                                               int j, double& o0, double& o1) {
    double mx[6][2], zc[6][2];
#pragma unroll
    for (int x = 0; x < 6; ++x) {
        mx[x][0] = mval(mu, dir, t[x], 0, J, j);
        mx[x][1] = mval(mu, dir, t[x], 1, J, j);
        zc[x][0] = Z[(int64_t)(2 * t[x]) * J + j];
        zc[x][1] = Z[(int64_t)(2 * t[x] + 1) * J + j];
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int x = 0; x < 6; ++x)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double p = mx[x][0] * zc[c][0] + mx[x][1] * zc[c][1];
            s0 += c_ref.Shat[x][a][c][0] * p;
            s1 += c_ref.Shat[x][a][c][1] * p;
        }
    o0 = g.det * (g.Ji[0][0] * s0 + g.Ji[1][0] * s1);
    o1 = g.det * (g.Ji[0][1] * s0 + g.Ji[1][1] * s1);
}

// Tw = C(W)^T mu_w, Tw1 = C(W1)^T mu_w, Tv = C(V)^T mu_v, Tv1 = C(V1)^T mu_v (per node, member)
__global__ void __launch_bounds__(kBlock) k_adj_T(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                                                  const int32_t* __restrict__ tri, const double* __restrict__ geo,
                                                  const uint8_t* __restrict__ dir, const double* __restrict__ muv,
                                                  const double* __restrict__ muw, const double* __restrict__ V,
                                                  const double* __restrict__ W, const double* __restrict__ V1,
                                                  const double* __restrict__ W1, double* __restrict__ Tv,
                                                  double* __restrict__ Tv1, double* __restrict__ Tw,
                                                  double* __restrict__ Tw1, int nP2, int J, int JP) {
    Lanes L = lanes(JP);
    const int64_t i = L.unit;
    if (i >= nP2) return;
    const int32_t q0 = inc_ptr[i], q1 = inc_ptr[i + 1];
    for (int j = L.j0; j < J; j += JP) {
        double a[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int32_t q = q0; q < q1; ++q) {
            const int64_t e = inc[q] >> 3;
            const int al = inc[q] & 7;
            int t[6];
#pragma unroll
            for (int x = 0; x < 6; ++x) t[x] = tri[e * 6 + x];
            Geo g = load_geo(geo, e);
            double o0, o1;
            conv_adj_local(t, g, al, muw, dir, W, J, j, o0, o1);
            a[0][0] += o0;
            a[0][1] += o1;
            conv_adj_local(t, g, al, muw, dir, W1, J, j, o0, o1);
            a[1][0] += o0;
            a[1][1] += o1;
            conv_adj_local(t, g, al, muv, dir, V, J, j, o0, o1);
            a[2][0] += o0;
            a[2][1] += o1;
            conv_adj_local(t, g, al, muv, dir, V1, J, j, o0, o1);
            a[3][0] += o0;
            a[3][1] += o1;
        }
        const int64_t o = (2 * i) * J + j;
        Tw[o] = a[0][0];
        Tw[o + J] = a[0][1];
        Tw1[o] = a[1][0];
        Tw1[o + J] = a[1][1];
        Tv[o] = a[2][0];
        Tv[o + J] = a[2][1];
        Tv1[o] = a[3][0];
        Tv1[o + J] = a[3][1];
    }
}

// Eddy term adjoint, per element (lanes over members): psi(e,q) = 2 mu dt |e| w_q
// sum_j grad mu_j(x_q) : grad X_j(x_q) and the maximiser j* of |z_j'(x_q)|^2;
// eta(e,q) = 2 psi z'_{j*}(x_q).
__global__ void __launch_bounds__(kBlock) k_adj_eddy(const int32_t* __restrict__ tri, const double* __restrict__ geo,
                                                     const uint8_t* __restrict__ dir, const double* __restrict__ Z,
                                                     const double* __restrict__ zbar, const double* __restrict__ mu,
                                                     const double* __restrict__ X, double* __restrict__ eta,
                                                     int32_t* __restrict__ jstar, int n_el, int J, int JP,
                                                     double eddy_c) {
    Lanes L = lanes(JP);
    const int64_t e = L.unit;
    const bool ok = e < n_el;
    double ps[7], bv[7], bz0[7], bz1[7];
    int bi[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        ps[q] = 0.0;
        bv[q] = -1.0;
        bi[q] = 0x7fffffff;
        bz0[q] = bz1[q] = 0.0;
    }
    Geo g{};
    int t[6] = {0, 0, 0, 0, 0, 0};
    if (ok) {
        g = load_geo(geo, e);
#pragma unroll
        for (int x = 0; x < 6; ++x) t[x] = tri[e * 6 + x];
        for (int j = L.j0; j < J; j += JP) {
            double m[6][2], xv[6][2], z[6][2];
#pragma unroll
            for (int x = 0; x < 6; ++x)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    m[x][c] = mval(mu, dir, t[x], c, J, j);
                    xv[x][c] = X[(int64_t)(2 * t[x] + c) * J + j];
                    z[x][c] = Z[(int64_t)(2 * t[x] + c) * J + j] - zbar[2 * t[x] + c];
                }
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                // reference gradients of mu_c and X_c, then physical: d/dx_d = sum_e' Ji[e'][d] d/dxi_e'
                double gm[2][2] = {{0, 0}, {0, 0}}, gx[2][2] = {{0, 0}, {0, 0}};
                double zq0 = 0.0, zq1 = 0.0;
#pragma unroll
                for (int x = 0; x < 6; ++x) {
                    const double d0 = c_ref.dphi[q][x][0], d1 = c_ref.dphi[q][x][1];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        gm[c][0] += m[x][c] * d0;
                        gm[c][1] += m[x][c] * d1;
                        gx[c][0] += xv[x][c] * d0;
                        gx[c][1] += xv[x][c] * d1;
                    }
                    zq0 += c_ref.phi[q][x] * z[x][0];
                    zq1 += c_ref.phi[q][x] * z[x][1];
                }
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const double pm = g.Ji[0][d] * gm[c][0] + g.Ji[1][d] * gm[c][1];
                        const double px = g.Ji[0][d] * gx[c][0] + g.Ji[1][d] * gx[c][1];
                        s += pm * px;
                    }
                ps[q] += s;
                const double mag = zq0 * zq0 + zq1 * zq1;
                if (mag > bv[q]) {   // members visited in increasing order: strict > keeps the lowest index
                    bv[q] = mag;
                    bi[q] = j;
                    bz0[q] = zq0;
                    bz1[q] = zq1;
                }
            }
        }
    }
    // butterflies over the member lanes: sum of psi, (max, lowest index) of |z'|^2
    for (int off = JP >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            ps[q] += __shfl_xor(ps[q], off, 64);
            const double ov = __shfl_xor(bv[q], off, 64);
            const int oi = __shfl_xor(bi[q], off, 64);
            const double o0 = __shfl_xor(bz0[q], off, 64);
            const double o1 = __shfl_xor(bz1[q], off, 64);
            if (ov > bv[q] || (ov == bv[q] && oi < bi[q])) {
                bv[q] = ov;
                bi[q] = oi;
                bz0[q] = o0;
                bz1[q] = o1;
            }
        }
    }
    if (ok && L.j0 == 0) {
        const double area = 0.5 * g.det;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double psi = eddy_c * area * c_ref.w[q] * ps[q];
            eta[(e * 7 + q) * 2] = 2.0 * psi * bz0[q];
            eta[(e * 7 + q) * 2 + 1] = 2.0 * psi * bz1[q];
            jstar[e * 7 + q] = bi[q];
        }
    }
}

// lambda for one variable at node i, member j (see file header)
__device__ __forceinline__ void adj_lambda_one(
    int64_t i, int j, int J, double inv_dt, double cp, double cm, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double* __restrict__ valM, const double* __restrict__ valK,
    const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc, const int32_t* __restrict__ tri,
    const double* __restrict__ geo, const uint8_t* __restrict__ dir, const double* __restrict__ mu_self,
    const double* __restrict__ mu_other, const double* __restrict__ Zc, const double* __restrict__ zcbar,
    const double* __restrict__ T, const double* __restrict__ Tbar, const double* __restrict__ T1bar,
    const double* __restrict__ eta, const int32_t* __restrict__ jstar, double invJ, double* __restrict__ lam,
    double* __restrict__ Kmu) {
    double mm0 = 0, mm1 = 0, km0 = 0, km1 = 0, ko0 = 0, ko1 = 0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int k = col[p];
        const double m = valM[p], kk = valK[p];
        const double s0 = mval(mu_self, dir, k, 0, J, j), s1 = mval(mu_self, dir, k, 1, J, j);
        const double o0 = mval(mu_other, dir, k, 0, J, j), o1 = mval(mu_other, dir, k, 1, J, j);
        mm0 += m * s0;
        mm1 += m * s1;
        km0 += kk * s0;
        km1 += kk * s1;
        ko0 += kk * o0;
        ko1 += kk * o1;
    }
    double l0 = mm0 * inv_dt - cp * km0 - cm * ko0;
    double l1 = mm1 * inv_dt - cp * km1 - cm * ko1;
    // N*(z_j') mu_self and the eddy gather over the incident elements
    for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
        const int64_t e = inc[q] >> 3;
        const int a = inc[q] & 7;
        Geo g = load_geo(geo, e);
        int t[6];
        double uh[6][2];
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            t[b] = tri[e * 6 + b];
            const double u0 = Zc[(int64_t)(2 * t[b]) * J + j] - zcbar[2 * t[b]];
            const double u1 = Zc[(int64_t)(2 * t[b] + 1) * J + j] - zcbar[2 * t[b] + 1];
            uh[b][0] = g.det * (g.Ji[0][0] * u0 + g.Ji[0][1] * u1);
            uh[b][1] = g.det * (g.Ji[1][0] * u0 + g.Ji[1][1] * u1);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double cf = 0.0;
#pragma unroll
            for (int b = 0; b < 6; ++b) cf += c_ref.Shat[a][b][c][0] * uh[b][0] + c_ref.Shat[a][b][c][1] * uh[b][1];
            l0 += cf * mval(mu_self, dir, t[c], 0, J, j);
            l1 += cf * mval(mu_self, dir, t[c], 1, J, j);
        }
#pragma unroll
        for (int qq = 0; qq < 7; ++qq) {
            const double f = c_ref.phi[qq][a] * ((jstar[e * 7 + qq] == j ? 1.0 : 0.0) - invJ);
            l0 -= f * eta[(e * 7 + qq) * 2];
            l1 -= f * eta[(e * 7 + qq) * 2 + 1];
        }
    }
    const int64_t o = (2 * i) * J + j;
    l0 += -T[o] + Tbar[2 * i] - T1bar[2 * i];
    l1 += -T[o + J] + Tbar[2 * i + 1] - T1bar[2 * i + 1];
    lam[o] = l0;
    lam[o + J] = l1;
    Kmu[o] = km0;
    Kmu[o + J] = km1;
}

__global__ void __launch_bounds__(kBlock) k_adj_lambda(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, const double* __restrict__ valM,
    const double* __restrict__ valK, const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
    const int32_t* __restrict__ tri, const double* __restrict__ geo, const uint8_t* __restrict__ dir,
    const double* __restrict__ coef, const double* __restrict__ muv, const double* __restrict__ muw,
    const double* __restrict__ V, const double* __restrict__ W, const double* __restrict__ vbar,
    const double* __restrict__ wbar, const double* __restrict__ Tv, const double* __restrict__ Tw,
    const double* __restrict__ Tvbar, const double* __restrict__ Tv1bar, const double* __restrict__ Twbar,
    const double* __restrict__ Tw1bar, const double* __restrict__ eta_v, const int32_t* __restrict__ js_v,
    const double* __restrict__ eta_w, const int32_t* __restrict__ js_w, double* __restrict__ lamV,
    double* __restrict__ lamW, double* __restrict__ Kmv, double* __restrict__ Kmw, int nP2, int J, int JP,
    double inv_dt) {
    Lanes L = lanes(JP);
    const int64_t i = L.unit;
    if (i >= nP2) return;
    const double invJ = 1.0 / J;
    for (int j = L.j0; j < J; j += JP) {
        const double cm = coef[j], cp = coef[J + j];
        // lambda_V: own v-problem (convection by w_j'), cross term from the w-problem,
        // T-terms of the w-problem, eddy term of S_w through l_v^2
        adj_lambda_one(i, j, J, inv_dt, cp, cm, rowptr, col, valM, valK, inc_ptr, inc, tri, geo, dir, muv, muw, W,
                       wbar, Tw, Twbar, Tw1bar, eta_v, js_v, invJ, lamV, Kmv);
        adj_lambda_one(i, j, J, inv_dt, cp, cm, rowptr, col, valM, valK, inc_ptr, inc, tri, geo, dir, muw, muv, V,
                       vbar, Tv, Tvbar, Tv1bar, eta_w, js_w, invJ, lamW, Kmw);
    }
}

// partial[(t*J + j) * nblk + block] = sum_r X_t[r, j] * Y_t[r(, j)] over the rows r < R
struct DotTask {
    const double* X[10];
    const double* Y[10];
    int yvec[10];       // 1: Y_t is an R-vector (same for all members)
    int nt;
};

__global__ void __launch_bounds__(kBlock) k_multidot(DotTask task, int64_t R, int J, int CW, double* __restrict__ partial) {
    __shared__ double red[kBlock];
    const int tx = threadIdx.x % CW, ty = threadIdx.x / CW, RG = kBlock / CW;
    const int j = blockIdx.y * CW + tx;
    const bool ok = ty < RG && j < J;
    double acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = 0.0;
    if (ok)
        for (int64_t r = (int64_t)blockIdx.x * RG + ty; r < R; r += (int64_t)gridDim.x * RG) {
#pragma unroll
            for (int t = 0; t < 10; ++t)
                if (t < task.nt) acc[t] += task.X[t][r * J + j] * (task.yvec[t] ? task.Y[t][r] : task.Y[t][r * J + j]);
        }
#pragma unroll
    for (int t = 0; t < 10; ++t) {
        if (t < task.nt) {
            red[threadIdx.x] = acc[t];
            __syncthreads();
            if (ty == 0 && ok) {
                double s = 0.0;
                for (int g2 = 0; g2 < RG; ++g2) s += red[g2 * CW + tx];
                partial[((int64_t)t * J + j) * gridDim.x + blockIdx.x] = s;
            }
            __syncthreads();
        }
    }
}

// gradient update (per member) from the 8 dot products
//   d = [av, bv, gv, aw, bw, gw, fv, fw]
__global__ void k_adj_grad(const double* __restrict__ d, int J, double* __restrict__ grad) {
    __shared__ double sums[4];
    if (threadIdx.x < 4) {
        const int idx[4] = {1, 2, 4, 5};
        double s = 0.0;
        for (int j = 0; j < J; ++j) s += d[idx[threadIdx.x] * J + j];
        sums[threadIdx.x] = s;
    }
    __syncthreads();
    const double common = (sums[0] - sums[1] + sums[2] - sums[3]) / (2.0 * J);
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
        const double av = d[j], bv = d[J + j], aw = d[3 * J + j], bw = d[4 * J + j];
        grad[3 * j] += -0.5 * av - 0.5 * bv - 0.5 * aw - 0.5 * bw + common;
        grad[3 * j + 1] += 0.5 * av - 0.5 * bv + 0.5 * aw - 0.5 * bw + common;
        grad[3 * j + 2] += d[6 * J + j] + d[7 * J + j];
    }
}

// lambda_j = (1/J) M zbar for every member (derivative of (1/2) ||<z>||_M^2)
__global__ void __launch_bounds__(kBlock) k_energy_adj(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                       const double* __restrict__ valM, const double* __restrict__ zbar,
                                                       double* __restrict__ lam, int nP2, int J, int JP) {
    Lanes L = lanes(JP);
    const int64_t i = L.unit;
    if (i >= nP2) return;
    double s0 = 0.0, s1 = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        s0 += valM[p] * zbar[2 * col[p]];
        s1 += valM[p] * zbar[2 * col[p] + 1];
    }
    for (int j = L.j0; j < J; j += JP) {
        lam[(2 * i) * J + j] = s0 / J;
        lam[(2 * i + 1) * J + j] = s1 / J;
    }
}

// out[i] = dir[i] ? 0 : M fhat (per component)
__global__ void __launch_bounds__(kBlock) k_mass_vec_masked(const int32_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ valM,
                                                            const uint8_t* __restrict__ dir,
                                                            const double* __restrict__ f, double* __restrict__ out,
                                                            int nP2) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nP2) return;
    double s0 = 0.0, s1 = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        s0 += valM[p] * f[2 * col[p]];
        s1 += valM[p] * f[2 * col[p] + 1];
    }
    out[2 * i] = dir[i] ? 0.0 : s0;
    out[2 * i + 1] = dir[i] ? 0.0 : s1;
}

// transposed operator values: A^T by the slot permutation; constant B/B^T exchange
__global__ void k_perm_A(const double* __restrict__ v, const int32_t* __restrict__ perm, double* __restrict__ vt,
                         float* __restrict__ vt32, int64_t nnz) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const double x = v[perm[p]];
    vt[p] = x;
    vt32[p] = (float)x;
}

__global__ void k_perm_B(const double* __restrict__ valB, const double* __restrict__ valBt,
                         const int32_t* __restrict__ permBtB, double* __restrict__ valB_T, double* __restrict__ valBt_T,
                         float* __restrict__ valB_T32, float* __restrict__ valBt_T32, int64_t nnzBt) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnzBt) return;
    const int64_t q = permBtB[p];
    for (int c = 0; c < 2; ++c) {
        valBt_T[2 * p + c] = valB[2 * q + c];
        valBt_T32[2 * p + c] = (float)valB[2 * q + c];
        valB_T[2 * q + c] = valBt[2 * p + c];
        valB_T32[2 * q + c] = (float)valBt[2 * p + c];
    }
}

// d = [pv_0 .. pv_{nm-1}, pw_0 .. pw_{nm-1}] (each J): mode projections of lambda_V^0, lambda_W^0;
// u-mode coefficients enter v and w with +1, B-mode coefficients with +-sqrt(s)
__global__ void k_ic_combine(const double* __restrict__ d, int nm, int J, double sq, double* __restrict__ g) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    for (int m = 0; m < nm; ++m) {
        const double pv = d[(int64_t)m * J + j], pw = d[(int64_t)(nm + m) * J + j];
        g[(int64_t)j * 2 * nm + m] = pv + pw;
        g[(int64_t)j * 2 * nm + nm + m] = sq * (pv - pw);
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_ic_combine(const double* d, int nm, int J, double sq, double* grad_ic, hipStream_t s) {
    hipLaunchKernelGGL(k_ic_combine, dim3((J + 63) / 64), dim3(64), 0, s, d, nm, J, sq, grad_ic);
    return hipGetLastError();
}

hipError_t launch_transpose_const(DevMesh& m, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_B, dim3((unsigned)((m.nnzBt + 255) / 256)), dim3(256), 0, s, m.valB, m.valBt, m.permBtB,
                       m.valB_T, m.valBt_T, m.valB_T32, m.valBt_T32, m.nnzBt);
    return hipGetLastError();
}

hipError_t launch_transpose_A(DevMesh& m, DevShared& S, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_A, dim3((unsigned)((m.nnzA + 255) / 256)), dim3(256), 0, s, S.valA, m.permA, S.valA_T,
                       S.valA_T32, m.nnzA);
    return hipGetLastError();
}

hipError_t launch_energy_adjoint(const DevMesh& m, const double* zbar, double* lam, int J, hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_energy_adj, dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, s, m.A_rowptr, m.A_col, m.valM, zbar,
                       lam, m.nP2, J, JP);
    return hipGetLastError();
}

hipError_t launch_mass_vec_masked(const DevMesh& m, const double* f, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_mass_vec_masked, dim3((m.nP2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m.A_rowptr, m.A_col,
                       m.valM, m.dir, f, out, m.nP2);
    return hipGetLastError();
}

hipError_t launch_adj_T(const DevMesh& m, const double* muv, const double* muw, const double* V, const double* W,
                        const double* V1, const double* W1, double* Tv, double* Tv1, double* Tw, double* Tw1, int J,
                        hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_adj_T, dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, s, m.inc_ptr, m.inc, m.tri, m.geo, m.dir,
                       muv, muw, V, W, V1, W1, Tv, Tv1, Tw, Tw1, m.nP2, J, JP);
    return hipGetLastError();
}

hipError_t launch_adj_eddy(const DevMesh& m, const double* Z, const double* zbar, const double* mu, const double* X,
                           double* eta, int32_t* jstar, int J, double eddy_c, hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_adj_eddy, dim3(grid_for(m.n_el, JP)), dim3(kBlock), 0, s, m.tri, m.geo, m.dir, Z, zbar, mu, X,
                       eta, jstar, m.n_el, J, JP, eddy_c);
    return hipGetLastError();
}

hipError_t launch_adj_lambda(const DevMesh& m, const double* coef, const double* muv, const double* muw, const double* V,
                             const double* W, const double* vbar, const double* wbar, const double* Tv,
                             const double* Tw, const double* Tvbar, const double* Tv1bar, const double* Twbar,
                             const double* Tw1bar, const double* eta_v, const int32_t* js_v, const double* eta_w,
                             const int32_t* js_w, double* lamV, double* lamW, double* Kmv, double* Kmw, int J,
                             double dt, hipStream_t s) {
    int JP = pick_jp(J);
    hipLaunchKernelGGL(k_adj_lambda, dim3(grid_for(m.nP2, JP)), dim3(kBlock), 0, s, m.A_rowptr, m.A_col, m.valM,
                       m.valK, m.inc_ptr, m.inc, m.tri, m.geo, m.dir, coef, muv, muw, V, W, vbar, wbar, Tv, Tw, Tvbar,
                       Tv1bar, Twbar, Tw1bar, eta_v, js_v, eta_w, js_w, lamV, lamW, Kmv, Kmw, m.nP2, J, JP, 1.0 / dt);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* const* X, const double* const* Y, const int* yvec, int nt, int64_t R, int J,
                           double* partial, double* out, hipStream_t s) {
    DotTask task{};
    task.nt = nt;
    for (int t = 0; t < nt; ++t) {
        task.X[t] = X[t];
        task.Y[t] = Y[t];
        task.yvec[t] = yvec[t];
    }
    int CW = pick_jp(J);
    int RG = kBlock / CW;
    int64_t need = (R + RG - 1) / RG;
    int nblk = (int)std::min<int64_t>(256, std::max<int64_t>(need, 1));
    hipLaunchKernelGGL(k_multidot, dim3(nblk, (J + CW - 1) / CW), dim3(kBlock), 0, s, task, R, J, CW, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_rows(partial, nblk, (int64_t)nt * J, out, s);
}

hipError_t launch_adj_grad(const double* d, int J, double* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_grad, dim3(1), dim3(256), 0, s, d, J, grad);
    return hipGetLastError();
}

}  // namespace mhd
