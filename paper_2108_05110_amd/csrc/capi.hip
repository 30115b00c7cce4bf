// C ABI of libmhd_ens: handle management, uploads, argument checks and the
// entry points declared in include/mhd_ens.h.  Every entry point validates its
// arguments on the host before it enqueues device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "device.h"

struct mhd_mesh_s {
    mhd::DevMesh d;
};
struct mhd_shared_s {
    mhd::DevShared d;
};
namespace mhd {
struct StepArgs {
    double *V, *W, *Q, *R;
    const double *f1, *f2, *gv, *gw;
    int J;
    bool operator==(const StepArgs& o) const {
        return V == o.V && W == o.W && Q == o.Q && R == o.R && f1 == o.f1 && f2 == o.f2 && gv == o.gv &&
               gw == o.gw && J == o.J;
    }
};

struct StepGraph {
    bool valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t stream = nullptr;
    StepArgs key{};
    mhd_solve_stats sv{}, sw{};
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        valid = false;
    }
};
}  // namespace mhd

struct mhd_group_s {
    std::vector<mhd_ctx> ctxs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
    mhd::StepGraph graph;
    std::vector<mhd::StepArgs> keys;
    std::vector<mhd_coeffs> coeffs;   // per context: dt, mu and mean viscosities baked into the graph
};

struct mhd_ctx_s {
    mhd::StepGraph graph;
    mhd_coeffs graph_coeffs{};
    std::vector<double> last_coef;          // member coefficients currently on the device
    mhd_mesh mesh = nullptr;
    mhd_shared Av = nullptr, Aw = nullptr;
    mhd_ctx_desc desc{};
    double *bv = nullptr, *bw = nullptr;    // right-hand sides (n x Jmax)
    double *Xv = nullptr, *Xw = nullptr;    // solution blocks [velocity; pressure]
    double* coef = nullptr;                 // 2 Jmax member coefficients
    hipStream_t side = nullptr;             // second stream: the w-subproblem of a fixed-schedule step
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double* host_coef = nullptr;            // pinned staging, 2 Jmax
    double* partial = nullptr;              // reductions
    double min_alpha = 0.0;                 // min_j alpha_j of the last step's parameters
    int warnings = 0;                       // MHD_WARN_ALPHA / MHD_WARN_MU of the last step's parameters
    // adjoint workspace (desc.adjoint)
    double *Tv = nullptr, *Tv1 = nullptr, *Tw = nullptr, *Tw1 = nullptr;   // (nP2,2,J)
    double *Kmv = nullptr, *Kmw = nullptr;                                  // (nP2,2,J)
    double* tmeans = nullptr;                                               // 4 x 2 nP2
    double *eta_v = nullptr, *eta_w = nullptr;                              // n_el x 7 x 2
    int32_t *js_v = nullptr, *js_w = nullptr;                               // n_el x 7
    double* Mf = nullptr;                                                   // 2 nP2
    double* dots = nullptr;                                                 // 10 J
    std::vector<void*> allocs;
};

namespace mhd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static std::atomic<int64_t> g_alloc_count{0}, g_alloc_bytes{0};

hipError_t dev_malloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
        g_alloc_count.fetch_add(1);
        g_alloc_bytes.fetch_add((int64_t)bytes);
    }
    return e;
}

namespace {

template <typename T>
mhd_status dev_alloc(std::vector<void*>& list, T** p, size_t count) {
    hipError_t e = dev_malloc((void**)p, std::max<size_t>(count * sizeof(T), 256));
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc(") + std::to_string(count * sizeof(T)) + "): " + hipGetErrorString(e));
        return MHD_ENOMEM;
    }
    list.push_back((void*)*p);
    return MHD_OK;
}

template <typename T>
mhd_status upload(std::vector<void*>& list, T** p, const std::vector<T>& h) {
    mhd_status rc = dev_alloc(list, p, h.size());
    if (rc) return rc;
    if (!h.empty()) MHD_HIP(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return MHD_OK;
}

mhd_status upload_csr(std::vector<void*>& list, DevCSR<double>& d, const HostCSR& h) {
    d.nrows = h.nrows;
    d.ncols = h.ncols;
    d.nnz = h.nnz();
    d.max_row = 0;
    for (size_t i = 0; i + 1 < h.rowptr.size(); ++i) d.max_row = std::max(d.max_row, h.rowptr[i + 1] - h.rowptr[i]);
    mhd_status rc;
    if ((rc = upload(list, &d.rowptr, h.rowptr))) return rc;
    if ((rc = upload(list, &d.col, h.col))) return rc;
    if ((rc = upload(list, &d.val, h.val))) return rc;
    std::vector<float> v32(h.val.begin(), h.val.end());
    if ((rc = upload(list, &d.val32, v32))) return rc;
    return MHD_OK;
}

// FP32 copy of a coarsest level's dense inverse with rows of ld floats, zero
// past column and row n (the matrix-core coarse solve reads 16 x 16 blocks)
std::vector<float> padded_inverse32(const HostLevel& H, int ld) {
    std::vector<float> c((size_t)ld * ld, 0.f);
    for (int r = 0; r < H.n; ++r)
        for (int k = 0; k < H.n; ++k) c[(size_t)r * ld + k] = (float)H.cinv[(size_t)r * H.n + k];
    return c;
}

void free_list(std::vector<void*>& list) {
    for (void* p : list) (void)hipFree(p);
    list.clear();
}

hipStream_t as_stream(mhd_stream_t s) { return (hipStream_t)s; }

#define CHECK_ARG(cond, msg)         \
    do {                             \
        if (!(cond)) {               \
            ::mhd::set_error(msg);   \
            return MHD_EINVAL;       \
        }                            \
    } while (0)

mhd_status build_device_mesh(DevMesh& D) {
    HostMesh& h = D.host;
    auto& L = D.allocs;
    D.nP2 = h.nP2;
    D.nP1 = h.nP1;
    D.n_el = h.n_el;
    D.n = 2 * (int64_t)h.nP2 + h.nP1;
    D.n_dir = (int)h.dir_nodes.size();
    D.pin = h.pin;
    RefTables t;
    make_ref_tables(t);
    upload_ref_tables(t);
    upload_ref_tables_adjoint(t);
    MHD_HIP(hipGetLastError());
    // element geometry: detJ and the inverse Jacobian of the affine map from the reference triangle
    std::vector<double> geo((size_t)h.n_el * 6, 0.0);
    for (int e = 0; e < h.n_el; ++e) {
        const double* p0 = &h.xy[2 * h.tri[(size_t)e * 6]];
        const double* p1 = &h.xy[2 * h.tri[(size_t)e * 6 + 1]];
        const double* p2 = &h.xy[2 * h.tri[(size_t)e * 6 + 2]];
        double a = p1[0] - p0[0], b = p2[0] - p0[0], c = p1[1] - p0[1], d = p2[1] - p0[1];
        double det = a * d - b * c;
        double* g = &geo[(size_t)e * 6];
        g[0] = det;
        g[1] = d / det;
        g[2] = -b / det;
        g[3] = -c / det;
        g[4] = a / det;
    }
    mhd_status rc;
    if ((rc = upload(L, &D.geo, geo))) return rc;
    if ((rc = upload(L, &D.xy, h.xy))) return rc;
    if ((rc = upload(L, &D.tri, h.tri))) return rc;
    if ((rc = upload(L, &D.tri1, h.tri1))) return rc;
    if ((rc = upload(L, &D.dir, h.dir))) return rc;
    std::vector<int32_t> dir_index(h.nP2, -1);
    for (size_t i = 0; i < h.dir_nodes.size(); ++i) dir_index[h.dir_nodes[i]] = (int32_t)i;
    if ((rc = upload(L, &D.dir_index, dir_index))) return rc;
    if ((rc = upload(L, &D.hs_p2, h.hs_p2))) return rc;
    if ((rc = upload(L, &D.cell_el, h.cell_el))) return rc;
    if ((rc = upload(L, &D.p1_of_p2, h.p1_of_p2))) return rc;
    D.nx = h.nx;
    D.ny = h.ny;
    if ((rc = upload(L, &D.dir_nodes, h.dir_nodes))) return rc;
    D.max_row = 0;
    for (const HostCSR* c : {&h.A, &h.Bt, &h.B})
        for (size_t i = 0; i + 1 < c->rowptr.size(); ++i)
            D.max_row = std::max(D.max_row, (int)(c->rowptr[i + 1] - c->rowptr[i]));
    D.max_row_bt = 0;
    for (size_t i = 0; i + 1 < h.Bt.rowptr.size(); ++i)
        D.max_row_bt = std::max(D.max_row_bt, (int)(h.Bt.rowptr[i + 1] - h.Bt.rowptr[i]));
    if ((rc = upload(L, &D.A_rowptr, h.A.rowptr))) return rc;
    if ((rc = upload(L, &D.A_col, h.A.col))) return rc;
    if ((rc = upload(L, &D.Bt_rowptr, h.Bt.rowptr))) return rc;
    if ((rc = upload(L, &D.Bt_col, h.Bt.col))) return rc;
    if ((rc = upload(L, &D.B_rowptr, h.B.rowptr))) return rc;
    if ((rc = upload(L, &D.B_col, h.B.col))) return rc;
    D.nnzA = h.A.nnz();
    D.nnzBt = h.Bt.nnz();
    D.nnzB = h.B.nnz();
    if ((rc = upload(L, &D.gA_ptr, h.gA_ptr))) return rc;
    if ((rc = upload(L, &D.gA_idx, h.gA_idx))) return rc;
    if ((rc = upload(L, &D.gB_ptr, h.gB_ptr))) return rc;
    if ((rc = upload(L, &D.gB_idx, h.gB_idx))) return rc;
    if ((rc = upload(L, &D.gBt_ptr, h.gBt_ptr))) return rc;
    if ((rc = upload(L, &D.gBt_idx, h.gBt_idx))) return rc;
    if ((rc = upload(L, &D.permA, h.permA))) return rc;
    if ((rc = upload(L, &D.permBtB, h.permBtB))) return rc;
    if ((rc = upload(L, &D.inc_ptr, h.inc_ptr))) return rc;
    if ((rc = upload(L, &D.inc, h.inc))) return rc;
    if ((rc = dev_alloc(L, &D.valM, D.nnzA))) return rc;
    if ((rc = dev_alloc(L, &D.valK, D.nnzA))) return rc;
    if ((rc = dev_alloc(L, &D.valB, 2 * D.nnzB))) return rc;
    if ((rc = dev_alloc(L, &D.valB32, 2 * D.nnzB))) return rc;
    if ((rc = dev_alloc(L, &D.valBt, 2 * D.nnzBt))) return rc;
    if ((rc = dev_alloc(L, &D.valBt32, 2 * D.nnzBt))) return rc;
    if ((rc = dev_alloc(L, &D.valB_T, 2 * D.nnzB))) return rc;
    if ((rc = dev_alloc(L, &D.valB_T32, 2 * D.nnzB))) return rc;
    if ((rc = dev_alloc(L, &D.valBt_T, 2 * D.nnzBt))) return rc;
    if ((rc = dev_alloc(L, &D.valBt_T32, 2 * D.nnzBt))) return rc;
    std::vector<double> dp(h.nP1, 0.0);
    if (h.pin >= 0) dp[h.pin] = 1.0;
    if ((rc = upload(L, &D.diagp, dp))) return rc;
    std::vector<float> dp32(dp.begin(), dp.end());
    if ((rc = upload(L, &D.diagp32, dp32))) return rc;
    if ((rc = upload(L, &D.mp, h.mp))) return rc;
    std::vector<double> mpi(h.mp.size());
    for (size_t i = 0; i < mpi.size(); ++i) mpi[i] = 1.0 / h.mp[i];
    if ((rc = upload(L, &D.mp_inv, mpi))) return rc;
    if ((rc = upload(L, &D.pfix, h.pfix))) return rc;
    if ((rc = dev_alloc(L, &D.scratch_coef, 2 * kMaxJ))) return rc;
    if ((rc = dev_alloc(L, &D.scratch_mean, 2 * (size_t)h.nP2))) return rc;
    // pressure multigrid hierarchy
    D.levels.resize(h.levels.size());
    D.levels_dt = h.schur_dt;
    D.levels_nuc = h.schur_nuc;
    for (size_t l = 0; l < h.levels.size(); ++l) {
        const HostLevel& H = h.levels[l];
        DevLevel& G = D.levels[l];
        G.n = H.n;
        G.omega = H.omega;
        if ((rc = upload_csr(L, G.L, H.L))) return rc;
        if ((rc = upload(L, &G.dinv, H.dinv))) return rc;
        std::vector<float> di32(H.dinv.begin(), H.dinv.end());
        if ((rc = upload(L, &G.dinv32, di32))) return rc;
        if (l + 1 < h.levels.size()) {
            if ((rc = upload_csr(L, G.P, H.P))) return rc;
            if ((rc = upload_csr(L, G.R, H.R))) return rc;
            if ((rc = upload_csr(L, G.Dn, H.Dn))) return rc;
            if ((rc = upload_csr(L, G.Up, H.Up))) return rc;
        } else {
            if ((rc = upload(L, &G.cinv, H.cinv))) return rc;
            G.ld32 = (H.n + 15) / 16 * 16;
            if ((rc = upload(L, &G.cinv32, padded_inverse32(H, G.ld32)))) return rc;
        }
    }
    // constant matrices (mass, stiffness, divergence) assembled on the device
    double* eb = nullptr;
    MHD_HIP(dev_malloc((void**)&eb, sizeof(double) * 108 * std::max(1, h.n_el)));
    hipError_t e = launch_const_assembly(D, eb, 0);
    if (e == hipSuccess) e = launch_transpose_const(D, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(eb);
    if (e != hipSuccess) {
        set_error(std::string("constant assembly: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    return MHD_OK;
}

mhd_status alloc_schur(DevShared& S);

mhd_status make_shared(DevMesh* m, int J_max, int restart, DevShared& S, bool compact) {
    S.mesh = m;
    S.Jmax = J_max;
    auto& L = S.allocs;
    mhd_status rc;
    if ((rc = dev_alloc(L, &S.valA, m->nnzA))) return rc;
    if ((rc = dev_alloc(L, &S.valA32, m->nnzA))) return rc;
    if ((rc = dev_alloc(L, &S.valA_T, m->nnzA))) return rc;
    if ((rc = dev_alloc(L, &S.valA_T32, m->nnzA))) return rc;
    if ((rc = dev_alloc(L, &S.dinvA, m->nP2))) return rc;
    if ((rc = dev_alloc(L, &S.dinvA32, m->nP2))) return rc;
    if ((rc = dev_alloc(L, &S.zbar, 2 * (size_t)m->nP2))) return rc;
    if ((rc = dev_alloc(L, &S.l2, 7 * (size_t)m->n_el))) return rc;
    if ((rc = dev_alloc(L, &S.elem, 36 * (size_t)m->n_el))) return rc;
    if ((rc = alloc_schur(S))) return rc;
    // defined values before the first assembly (the kernel tuner may run on them)
    MHD_HIP(hipMemset(S.valA, 0, sizeof(double) * (size_t)m->nnzA));
    MHD_HIP(hipMemset(S.valA32, 0, sizeof(float) * (size_t)m->nnzA));
    MHD_HIP(hipMemset(S.dinvA, 0, sizeof(double) * (size_t)m->nP2));
    MHD_HIP(hipMemset(S.dinvA32, 0, sizeof(float) * (size_t)m->nP2));
    return alloc_gmres(S, restart, compact);
}

void free_shared(DevShared& S) {
    free_list(S.allocs);
    if (S.gw.host_res) (void)hipHostFree(S.gw.host_res);
    S.gw.host_res = nullptr;
}

mhd_status check_coeffs(const mhd_coeffs* c) {
    CHECK_ARG(c, "null coefficients");
    CHECK_ARG(std::isfinite(c->dt) && c->dt > 0, "dt must be positive and finite");
    CHECK_ARG(std::isfinite(c->mu) && c->mu >= 0, "mu must be non-negative");
    CHECK_ARG(std::isfinite(c->nu_bar) && c->nu_bar >= 0, "nu_bar must be non-negative");
    CHECK_ARG(std::isfinite(c->num_bar) && c->num_bar >= 0, "num_bar must be non-negative");
    CHECK_ARG(c->convective == 0 || c->convective == 1, "convective must be 0 or 1");
    return MHD_OK;
}

// The handle's Schur-approximation values for (dt, nu_c): recomputed on the host
// (the mesh keeps the last computation) and copied into the handle's own value
// arrays when its key changes.  Synchronous; never called under capture.
mhd_status refresh_schur(DevShared& S, double dt, double nu_c) {
    if (S.schur_dt == dt && S.schur_nuc == nu_c) return MHD_OK;
    DevMesh& D = *S.mesh;
    HostMesh& h = D.host;
    if (!(h.schur_dt == dt && h.schur_nuc == nu_c)) {
        mhd_status rc = schur_values(h, dt, nu_c);
        if (rc) return rc;
    }
    MHD_HIP(hipDeviceSynchronize());
    for (size_t l = 0; l < h.levels.size(); ++l) {
        const HostLevel& H = h.levels[l];
        DevLevel& G = S.levels[l];
        if ((int64_t)H.L.val.size() != G.L.nnz) {
            set_error("refresh_schur: pattern size mismatch");
            return MHD_EINVAL;
        }
        G.omega = H.omega;
        std::vector<float> v32(H.L.val.begin(), H.L.val.end());
        std::vector<float> d32(H.dinv.begin(), H.dinv.end());
        MHD_HIP(hipMemcpy(G.L.val, H.L.val.data(), sizeof(double) * H.L.val.size(), hipMemcpyHostToDevice));
        MHD_HIP(hipMemcpy(G.L.val32, v32.data(), sizeof(float) * v32.size(), hipMemcpyHostToDevice));
        MHD_HIP(hipMemcpy(G.dinv, H.dinv.data(), sizeof(double) * H.dinv.size(), hipMemcpyHostToDevice));
        MHD_HIP(hipMemcpy(G.dinv32, d32.data(), sizeof(float) * d32.size(), hipMemcpyHostToDevice));
        for (auto hd : {std::make_pair(&H.Dn, &G.Dn), std::make_pair(&H.Up, &G.Up)}) {
            const HostCSR& hc = *hd.first;
            DevCSR<double>& dc = *hd.second;
            if (hc.nnz() == 0) continue;
            if (hc.nnz() != dc.nnz) {
                set_error("refresh_schur: fused pattern size mismatch");
                return MHD_EINVAL;
            }
            std::vector<float> f32(hc.val.begin(), hc.val.end());
            MHD_HIP(hipMemcpy(dc.val, hc.val.data(), sizeof(double) * hc.val.size(), hipMemcpyHostToDevice));
            MHD_HIP(hipMemcpy(dc.val32, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice));
        }
        if (l + 1 == h.levels.size()) {
            const std::vector<float> c32 = padded_inverse32(H, G.ld32);
            MHD_HIP(hipMemcpy(G.cinv, H.cinv.data(), sizeof(double) * H.cinv.size(), hipMemcpyHostToDevice));
            MHD_HIP(hipMemcpy(G.cinv32, c32.data(), sizeof(float) * c32.size(), hipMemcpyHostToDevice));
        }
    }
    S.schur_dt = dt;
    S.schur_nuc = nu_c;
    return MHD_OK;
}

// value arrays of a handle's hierarchy: the mesh's patterns, own values (a copy
// of the mesh's current ones until the first refresh)
mhd_status alloc_schur(DevShared& S) {
    DevMesh& D = *S.mesh;
    auto& L = S.allocs;
    S.levels = D.levels;
    mhd_status rc;
    auto dup = [&](auto** p, const auto* src, size_t count) -> mhd_status {
        mhd_status r = dev_alloc(L, p, count);
        if (r) return r;
        if (count) MHD_HIP(hipMemcpy(*p, src, sizeof(**p) * count, hipMemcpyDeviceToDevice));
        return MHD_OK;
    };
    for (size_t l = 0; l < D.levels.size(); ++l) {
        const DevLevel& M = D.levels[l];
        DevLevel& G = S.levels[l];
        if ((rc = dup(&G.L.val, M.L.val, M.L.nnz))) return rc;
        if ((rc = dup(&G.L.val32, M.L.val32, M.L.nnz))) return rc;
        if ((rc = dup(&G.dinv, M.dinv, M.n))) return rc;
        if ((rc = dup(&G.dinv32, M.dinv32, M.n))) return rc;
        if (M.Dn.nnz) {
            if ((rc = dup(&G.Dn.val, M.Dn.val, M.Dn.nnz))) return rc;
            if ((rc = dup(&G.Dn.val32, M.Dn.val32, M.Dn.nnz))) return rc;
        }
        if (M.Up.nnz) {
            if ((rc = dup(&G.Up.val, M.Up.val, M.Up.nnz))) return rc;
            if ((rc = dup(&G.Up.val32, M.Up.val32, M.Up.nnz))) return rc;
        }
        if (l + 1 == D.levels.size()) {
            if ((rc = dup(&G.cinv, M.cinv, (size_t)M.n * M.n))) return rc;
            if ((rc = dup(&G.cinv32, M.cinv32, (size_t)M.ld32 * M.ld32))) return rc;
        }
    }
    // the key of the values just copied: the mesh's device values keep the
    // parameters they were built for, while its host copy follows the last refresh
    S.schur_dt = D.levels_dt;
    S.schur_nuc = D.levels_nuc;
    return MHD_OK;
}

mhd_status assemble_shared_impl(DevMesh& m, const mhd_coeffs& c, const double* z, int J, DevShared& S, hipStream_t s) {
    mhd_status rc = refresh_schur(S, c.dt, 0.5 * (c.nu_bar + c.num_bar));
    if (rc) return rc;
    hipError_t e = launch_mean(z, S.zbar, 2 * (int64_t)m.nP2, J, s);
    if (e == hipSuccess) e = launch_eddy_l2(m, z, S.zbar, S.l2, J, s);
    if (e == hipSuccess) e = launch_assemble_A(m, c, S.zbar, S.l2, S.elem, S.valA, S.valA32, S.dinvA, S.dinvA32, s);
    if (e == hipSuccess) e = scatter_ell_values(S, s);
    if (e != hipSuccess) {
        set_error(std::string("assemble_shared: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    S.coeffs = c;
    S.assembled = true;
    return MHD_OK;
}

mhd_status check_solver_opts(const mhd_solver_opts* o) {
    CHECK_ARG(o, "null solver options");
    CHECK_ARG(o->precision == MHD_FP64 || o->precision == MHD_FP32_IR, "precision must be MHD_FP64 or MHD_FP32_IR");
    CHECK_ARG(std::isfinite(o->rtol) && o->rtol > 0 && o->rtol < 1, "rtol must be in (0,1)");
    CHECK_ARG(std::isfinite(o->inner_rtol) && o->inner_rtol > 0 && o->inner_rtol < 1, "inner_rtol must be in (0,1)");
    CHECK_ARG(o->maxit >= 1, "maxit must be >= 1");
    CHECK_ARG(o->restart >= 1 && o->restart <= kMaxRestart, "restart must be in [1, 40]");
    CHECK_ARG(o->jacobi_sweeps >= 1 && o->jacobi_sweeps <= 16, "jacobi_sweeps must be in [1, 16]");
    CHECK_ARG(o->cgs_passes >= 0 && o->cgs_passes <= 3, "cgs_passes must be 0, 1, 2 or 3");
    CHECK_ARG(o->fixed_cycles >= 0 && o->fixed_cycles <= 64, "fixed_cycles must be in [0, 64]");
    CHECK_ARG(o->jacobi_omega == 0 || (std::isfinite(o->jacobi_omega) && o->jacobi_omega > 0 && o->jacobi_omega <= 1.5),
              "jacobi_omega must be 0 (default) or in (0, 1.5]");
    CHECK_ARG(o->mg_unfused == 0 || o->mg_unfused == 1, "mg_unfused must be 0 or 1");
    CHECK_ARG(o->mg_cycles >= 0 && o->mg_cycles <= 2, "mg_cycles must be 0, 1 or 2");
    CHECK_ARG(o->block_krylov == 0 || (o->block_krylov == 1 && o->fixed_cycles == 0),
              "block_krylov must be 0, or 1 with the adaptive schedule (fixed_cycles 0)");
    CHECK_ARG(o->keep_converged == 0 || o->keep_converged == 1, "keep_converged must be 0 or 1");
    CHECK_ARG(o->mg_post >= 0 && o->mg_post <= 8, "mg_post must be in [0, 8]");
    return MHD_OK;
}

// host part of a step: mean viscosities, member coefficients (uploaded when they
// change), Schur-hierarchy refresh; no device work is left pending on the
// pinned staging buffer when it is rewritten
mhd_status step_prepare(mhd_ctx ctx, const mhd_step_inputs* in, mhd_coeffs& c, hipStream_t st) {
    CHECK_ARG(in->nu && in->nu_m, "mhd_ens_step: null nu / nu_m");
    const int J = in->J;
    if (J < 1 || J > ctx->desc.J_max) {
        set_error("mhd_ens_step: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    DevMesh& D = ctx->mesh->d;
    CHECK_ARG((in->g_v && in->g_w) || D.n_dir == 0, "mhd_ens_step: null Dirichlet data");
    double nub = 0, numb = 0;
    for (int j = 0; j < J; ++j) {
        CHECK_ARG(std::isfinite(in->nu[j]) && std::isfinite(in->nu_m[j]), "mhd_ens_step: non-finite nu");
        nub += in->nu[j];
        numb += in->nu_m[j];
    }
    nub /= J;
    numb /= J;
    // stability conditions of Section 3.1: alpha_j = nu_bar + num_bar - |nu_j - nu_m,j|
    // - |nu_j' + nu_m,j'| > 0 for every member and mu > 1/2; the scheme runs either way
    double amin = INFINITY;
    for (int j = 0; j < J; ++j)
        amin = std::min(amin, nub + numb - std::fabs(in->nu[j] - in->nu_m[j]) -
                                  std::fabs((in->nu[j] - nub) + (in->nu_m[j] - numb)));
    ctx->min_alpha = amin;
    ctx->warnings = (amin > 0 ? 0 : MHD_WARN_ALPHA) | (ctx->desc.coeffs.mu > 0.5 ? 0 : MHD_WARN_MU);
    std::vector<double> cf(2 * (size_t)J);
    for (int j = 0; j < J; ++j) {
        cf[j] = 0.5 * (in->nu[j] - in->nu_m[j]);
        cf[J + j] = 0.5 * ((in->nu[j] - nub) + (in->nu_m[j] - numb));
    }
    if (cf != ctx->last_coef) {
        MHD_HIP(hipStreamSynchronize(st));
        std::copy(cf.begin(), cf.end(), ctx->host_coef);
        MHD_HIP(hipMemcpyAsync(ctx->coef, ctx->host_coef, sizeof(double) * 2 * J, hipMemcpyHostToDevice, st));
        ctx->last_coef = cf;
    }
    c = ctx->desc.coeffs;
    c.nu_bar = nub;
    c.num_bar = numb;
    if (ctx->desc.graph && ctx->graph.valid) {
        const mhd_coeffs& g = ctx->graph_coeffs;
        if (g.dt != c.dt || g.nu_bar != c.nu_bar || g.num_bar != c.num_bar || g.mu != c.mu) ctx->graph.reset();
    }
    ctx->graph_coeffs = c;
    mhd_status rc = refresh_schur(ctx->Av->d, c.dt, 0.5 * (c.nu_bar + c.num_bar));
    if (rc == MHD_OK) rc = refresh_schur(ctx->Aw->d, c.dt, 0.5 * (c.nu_bar + c.num_bar));
    return rc;
}

// device part of a step (a1-a6): capturable into a graph when the solver runs a fixed schedule
// One subproblem of a step on stream st: shared matrix from the other
// variable, right-hand sides, solve into X (initial guess: the state at n).
mhd_status subproblem(mhd_ctx ctx, const mhd_coeffs& c, int J, const double* self, const double* other,
                      const double* pres, const double* f, const double* g, DevShared& A, double* rhs,
                      double* X, hipStream_t st, mhd_solve_stats* stats) {
    DevMesh& D = ctx->mesh->d;
    mhd_status rc;
    if ((rc = assemble_shared_impl(D, c, other, J, A, st))) return rc;
    hipError_t e = launch_rhs_strip(D, c, J, self, other, A.zbar, ctx->coef, f, g, rhs, MHD_FP64, st);
    if (e != hipSuccess) {
        set_error(std::string("mhd_ens_step rhs: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    const size_t vel = sizeof(double) * 2 * (size_t)D.nP2 * J;
    const size_t prs = sizeof(double) * (size_t)D.nP1 * J;
    MHD_HIP(hipMemcpyAsync(X, self, vel, hipMemcpyDeviceToDevice, st));
    MHD_HIP(hipMemcpyAsync(X + 2 * (int64_t)D.nP2 * J, pres, prs, hipMemcpyDeviceToDevice, st));
    return solve_shared(A, rhs, X, J, ctx->desc.solver, stats, st);
}

// device part of a step (a1-a6): capturable into a graph when the solver runs
// a fixed schedule.  Both subproblems read time level n only; with a fixed
// schedule and `split`, the w-subproblem runs on the context's second stream,
// forked from and joined back into stv.  The new state is written after both.
mhd_status step_device(mhd_ctx ctx, const mhd_coeffs& c, const StepArgs& a, hipStream_t stv, mhd_solve_stats* sv,
                       mhd_solve_stats* sw, bool split) {
    DevMesh& D = ctx->mesh->d;
    const int J = a.J;
    const bool two = split && ctx->side != nullptr;
    hipStream_t stw = two ? ctx->side : stv;
    if (two) {
        MHD_HIP(hipEventRecord(ctx->ev_fork, stv));
        MHD_HIP(hipStreamWaitEvent(stw, ctx->ev_fork, 0));
    }
    // v-problem convected by <w>, w-problem by <v>
    mhd_status rv = subproblem(ctx, c, J, a.V, a.W, a.Q, a.f1, a.gv, ctx->Av->d, ctx->bv, ctx->Xv, stv, sv);
    if (rv != MHD_OK && rv != MHD_ENOCONV) return rv;
    mhd_status rw =
        subproblem(ctx, c, J, a.W, a.V, a.R, a.f2, a.gw, ctx->Aw->d, ctx->bw, ctx->Xw, stw, sw);
    if (rw != MHD_OK && rw != MHD_ENOCONV) return rw;
    if (two) {
        MHD_HIP(hipEventRecord(ctx->ev_join, stw));
        MHD_HIP(hipStreamWaitEvent(stv, ctx->ev_join, 0));
    }
    const size_t vel = sizeof(double) * 2 * (size_t)D.nP2 * J;
    const size_t prs = sizeof(double) * (size_t)D.nP1 * J;
    const int64_t poff = 2 * (int64_t)D.nP2 * J;
    MHD_HIP(hipMemcpyAsync(a.V, ctx->Xv, vel, hipMemcpyDeviceToDevice, stv));
    MHD_HIP(hipMemcpyAsync(a.Q, ctx->Xv + poff, prs, hipMemcpyDeviceToDevice, stv));
    MHD_HIP(hipMemcpyAsync(a.W, ctx->Xw, vel, hipMemcpyDeviceToDevice, stv));
    MHD_HIP(hipMemcpyAsync(a.R, ctx->Xw + poff, prs, hipMemcpyDeviceToDevice, stv));
    if (D.pin >= 0) {
        hipError_t e = launch_pressure_zero_mean(D, a.Q, J, ctx->partial, stv);
        if (e == hipSuccess) e = launch_pressure_zero_mean(D, a.R, J, ctx->partial, stv);
        if (e != hipSuccess) {
            set_error(std::string("pressure normalisation: ") + hipGetErrorString(e));
            return MHD_EHIP;
        }
    }
    return (rv == MHD_ENOCONV || rw == MHD_ENOCONV) ? MHD_ENOCONV : MHD_OK;
}

// E = (||<v>||^2 + ||<w>||^2)/2 with the P2 mass matrix (synchronises)
mhd_status step_energy(mhd_ctx ctx, const StepArgs& a, hipStream_t stv, double* energy) {
    DevMesh& D = ctx->mesh->d;
    double* zb = ctx->Av->d.zbar;
    double E = 0.0;
    int nblk = (D.nP2 + 255) / 256;
    std::vector<double> hp(nblk);
    for (int var = 0; var < 2; ++var) {
        hipError_t e = launch_mean(var == 0 ? a.V : a.W, zb, 2 * (int64_t)D.nP2, a.J, stv);
        if (e == hipSuccess) e = launch_energy_partial(D, zb, ctx->partial, stv);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hp.data(), ctx->partial, sizeof(double) * nblk, hipMemcpyDeviceToHost, stv);
        if (e == hipSuccess) e = hipStreamSynchronize(stv);
        if (e != hipSuccess) {
            set_error(std::string("energy: ") + hipGetErrorString(e));
            return MHD_EHIP;
        }
        for (double v : hp) E += v;
    }
    *energy = 0.5 * E;
    return MHD_OK;
}

// Right-hand sides of one subproblem (a3): member coefficients c-, c+ and the
// ensemble mean of the other variable into the given device scratch, then the
// node kernel.
mhd_status check_rhs_args(const char* who, mhd_mesh m, const mhd_coeffs* c, int which, int J, const double* self_n,
                          const double* other_n, const double* nu, const double* nu_m, const double* bc_vals,
                          const void* rhs, int precision) {
    if (!m) {
        set_error(std::string(who) + ": null mesh");
        return MHD_EINVAL;
    }
    mhd_status rc = check_coeffs(c);
    if (rc) return rc;
    if (!(which == MHD_V_PROBLEM || which == MHD_W_PROBLEM)) {
        set_error(std::string(who) + ": which must be V or W");
        return MHD_EINVAL;
    }
    if (J < 1 || J > kMaxJ) {
        set_error(std::string(who) + ": J must be in [1, 4096]");
        return MHD_EINVAL;
    }
    if (!(self_n && other_n && nu && nu_m && rhs)) {
        set_error(std::string(who) + ": null array");
        return MHD_EINVAL;
    }
    if (!bc_vals && m->d.n_dir != 0) {
        set_error(std::string(who) + ": null bc_vals with Dirichlet nodes");
        return MHD_EINVAL;
    }
    if (precision != MHD_FP64 && precision != MHD_FP32_IR) {
        set_error(std::string(who) + ": precision must be MHD_FP64 or MHD_FP32_IR");
        return MHD_EINVAL;
    }
    return MHD_OK;
}

mhd_status assemble_rhs_impl(const char* who, DevMesh& D, const mhd_coeffs& c, int J, const double* self_n,
                             const double* other_n, const double* nu, const double* nu_m, const double* forcing,
                             const double* bc_vals, void* rhs, int precision, double* coef, double* mean,
                             hipStream_t st) {
    hipError_t e = launch_member_coefs(nu, nu_m, J, coef, st);
    if (e == hipSuccess) e = launch_mean(other_n, mean, 2 * (int64_t)D.nP2, J, st);
    if (e == hipSuccess)
        e = launch_rhs_strip(D, c, J, self_n, other_n, mean, coef, forcing, bc_vals, rhs, precision, st);
    if (e != hipSuccess) {
        set_error(std::string(who) + ": " + hipGetErrorString(e));
        return MHD_EHIP;
    }
    return MHD_OK;
}

// Fixed device scratch of the allocation-free right-hand side call: 2 J member
// coefficients, then (at a 256-byte boundary) the 2 nP2 values of the ensemble
// mean.  4 Mi doubles (32 MiB) per device cover J <= 4096 with nP2 <= 2,093,056
// (the 1022 x 1022 unit square).  In host code `scratch` names a host-side
// stand-in, never the device memory: every host use goes through the address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchDoubles = size_t(4) << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

size_t noalloc_mean_offset(int J) { return ((2 * (size_t)J + 31) / 32) * 32; }
size_t noalloc_rhs_doubles(int J, int64_t nP2) { return noalloc_mean_offset(J) + 2 * (size_t)nP2; }

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

// device address of `scratch` on the current device, looked up once per device
mhd_status scratch_base(const char* who, double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) {
        set_error(std::string(who) + ": hipGetDevice: " + hipGetErrorString(e));
        return MHD_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string(who) + ": hipGetSymbolAddress(scratch): " + hipGetErrorString(e));
            return MHD_EHIP;
        }
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}

// A C++ exception (host allocation failure inside a container, for example)
// must not cross the C ABI: every entry point turns it into a status.
mhd_status exception_status() {
    try {
        throw;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return MHD_ENOMEM;
    } catch (const std::exception& ex) {
        set_error(std::string("internal error: ") + ex.what());
        return MHD_EINVAL;
    } catch (...) {
        set_error("internal error");
        return MHD_EINVAL;
    }
}

}  // namespace
}  // namespace mhd

using namespace mhd;

extern "C" {

const char* mhd_ens_last_error(void) { return g_last_error.c_str(); }

const char* mhd_ens_version(void) { return "mhd_ens 0.1 (gfx950)"; }

mhd_status mhd_ens_mesh_counts(const mhd_mesh_desc* d, mhd_mesh_info* info) try {
    CHECK_ARG(info, "mhd_ens_mesh_counts: null info");
    HostMesh m;
    mhd_status rc = build_mesh(d, m, true);
    if (rc) return rc;
    mesh_counts(m, info);
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_mesh(const mhd_mesh_desc* d, mhd_mesh* out, mhd_mesh_info* info) try {
    CHECK_ARG(out, "mhd_ens_mesh: null output handle");
    *out = nullptr;
    mhd_mesh m = new (std::nothrow) mhd_mesh_s;
    if (!m) {
        set_error("mhd_ens_mesh: host allocation failed");
        return MHD_ENOMEM;
    }
    mhd_status rc = build_mesh(d, m->d.host, true);
    if (rc == MHD_OK) rc = build_device_mesh(m->d);
    if (rc != MHD_OK) {
        free_list(m->d.allocs);
        delete m;
        return rc;
    }
    if (info) mesh_counts(m->d.host, info);
    *out = m;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_mesh_coords(mhd_mesh m, double* xy_p2, int32_t* dir_nodes) try {
    CHECK_ARG(m, "mhd_ens_mesh_coords: null mesh");
    if (xy_p2) std::memcpy(xy_p2, m->d.host.xy.data(), sizeof(double) * m->d.host.xy.size());
    if (dir_nodes)
        std::memcpy(dir_nodes, m->d.host.dir_nodes.data(), sizeof(int32_t) * m->d.host.dir_nodes.size());
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_mesh_elements(mhd_mesh m, int32_t* tri) try {
    CHECK_ARG(m && tri, "mhd_ens_mesh_elements: null argument");
    std::memcpy(tri, m->d.host.tri.data(), sizeof(int32_t) * m->d.host.tri.size());
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_mesh_free(mhd_mesh m) try {
    if (!m) return MHD_OK;
    free_list(m->d.allocs);
    for (auto*& t : m->d.tiling) {
        delete t;
        t = nullptr;
    }
    for (auto*& t : m->d.ell) {
        delete t;
        t = nullptr;
    }
    delete m;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

// compact: with the buffers of the adaptive solver's member compaction
mhd_status shared_create(mhd_mesh m, int J_max, int restart, bool compact, mhd_shared* out);

mhd_status mhd_ens_shared_create(mhd_mesh m, int J_max, int restart, mhd_shared* out) try {
    return shared_create(m, J_max, restart, true, out);
} catch (...) {
    return exception_status();
}

mhd_status shared_create(mhd_mesh m, int J_max, int restart, bool compact, mhd_shared* out) {
    CHECK_ARG(out, "mhd_ens_shared_create: null output handle");
    *out = nullptr;
    CHECK_ARG(m, "mhd_ens_shared_create: null mesh");
    CHECK_ARG(J_max >= 1 && J_max <= kMaxJ, "mhd_ens_shared_create: J_max must be in [1, 4096]");
    CHECK_ARG(restart >= 1 && restart <= kMaxRestart, "mhd_ens_shared_create: restart must be in [1, 40]");
    mhd_shared A = new (std::nothrow) mhd_shared_s;
    if (!A) return MHD_ENOMEM;
    mhd_status rc = make_shared(&m->d, J_max, restart, A->d, compact);
    if (rc) {
        free_shared(A->d);
        delete A;
        return rc;
    }
    *out = A;
    return MHD_OK;
}

mhd_status mhd_ens_shared_free(mhd_shared A) try {
    if (!A) return MHD_OK;
    free_shared(A->d);
    delete A;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_assemble_shared(mhd_mesh m, const mhd_coeffs* c, const double* z_other, int J, mhd_shared A,
                                   mhd_stream_t s) try {
    CHECK_ARG(m && A, "mhd_ens_assemble_shared: null handle");
    CHECK_ARG(A->d.mesh == &m->d, "mhd_ens_assemble_shared: shared handle belongs to another mesh");
    CHECK_ARG(z_other, "mhd_ens_assemble_shared: null z_other");
    mhd_status rc = check_coeffs(c);
    if (rc) return rc;
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_assemble_shared: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    return assemble_shared_impl(m->d, *c, z_other, J, A->d, as_stream(s));
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_shared_csr(mhd_shared A, mhd_csr_view* v) try {
    CHECK_ARG(A && v, "mhd_ens_shared_csr: null argument");
    DevMesh& m = *A->d.mesh;
    v->rowptr_A = m.A_rowptr;
    v->col_A = m.A_col;
    v->val_A = A->d.valA;
    v->val_A32 = A->d.valA32;
    v->rowptr_Bt = m.Bt_rowptr;
    v->col_Bt = m.Bt_col;
    v->val_Bt = m.valBt;
    v->rowptr_B = m.B_rowptr;
    v->col_B = m.B_col;
    v->val_B = m.valB;
    v->diag_p = m.diagp;
    v->nP2 = m.nP2;
    v->nP1 = m.nP1;
    v->nnz_A = m.nnzA;
    v->nnz_Bt = m.nnzBt;
    v->nnz_B = m.nnzB;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_assemble_rhs(mhd_mesh m, const mhd_coeffs* c, int which, int J, const double* self_n,
                                const double* other_n, const double* nu, const double* nu_m, const double* forcing,
                                const double* bc_vals, void* rhs, int precision, mhd_stream_t s) try {
    mhd_status rc = check_rhs_args("mhd_ens_assemble_rhs", m, c, which, J, self_n, other_n, nu, nu_m, bc_vals, rhs,
                                   precision);
    if (rc) return rc;
    DevMesh& D = m->d;
    return assemble_rhs_impl("mhd_ens_assemble_rhs", D, *c, J, self_n, other_n, nu, nu_m, forcing, bc_vals, rhs,
                             precision, D.scratch_coef, D.scratch_mean, as_stream(s));
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_assemble_rhs_noalloc(mhd_mesh m, const mhd_coeffs* c, int which, int J, const double* self_n,
                                        const double* other_n, const double* nu, const double* nu_m,
                                        const double* forcing, const double* bc_vals, void* rhs, int precision,
                                        mhd_stream_t s) try {
    static const char* who = "mhd_ens_assemble_rhs_noalloc";
    mhd_status rc = check_rhs_args(who, m, c, which, J, self_n, other_n, nu, nu_m, bc_vals, rhs, precision);
    if (rc) return rc;
    DevMesh& D = m->d;
    const size_t need = noalloc_rhs_doubles(J, D.nP2);
    if (need > kScratchDoubles) {
        set_error(std::string(who) + ": needs " + std::to_string(need * sizeof(double)) +
                  " bytes of scratch (2 J member coefficients + 2 nP2 mean values), more than the fixed " +
                  std::to_string(kScratchDoubles * sizeof(double)) + "-byte device array");
        return MHD_ESHAPE;
    }
    double* base = nullptr;
    if ((rc = scratch_base(who, &base))) return rc;
    double* coef = base;
    double* mean = base + noalloc_mean_offset(J);
    return assemble_rhs_impl(who, D, *c, J, self_n, other_n, nu, nu_m, forcing, bc_vals, rhs, precision, coef,
                             mean, as_stream(s));
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_solve(mhd_shared A, const double* rhs, double* x, int J, const mhd_solver_opts* o,
                         mhd_solve_stats* st, mhd_stream_t s) try {
    CHECK_ARG(A, "mhd_ens_solve: null handle");
    CHECK_ARG(rhs && x, "mhd_ens_solve: null array");
    mhd_status rc = check_solver_opts(o);
    if (rc) return rc;
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_solve: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    CHECK_ARG(o->restart <= A->d.gw.restart, "mhd_ens_solve: restart larger than the handle's");
    CHECK_ARG(A->d.assembled, "mhd_ens_solve: matrix not assembled");
    CHECK_ARG(!o->block_krylov || ((J == 16 || J == 32 || J == 64 || J == 128) && A->d.gw.bmat),
              "mhd_ens_solve: block GMRES needs J in {16, 32, 64, 128} (and J_max <= 128)");
    hipStream_t hs = as_stream(s);
    rc = solve_shared(A->d, rhs, x, J, *o, st, hs);
    if (rc || !st || o->fixed_cycles == 0) return rc;
    // fixed schedule: the residuals were not looked at during the solve
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MHD_HIP(hipStreamIsCapturing(hs, &cs));
    if (cs != hipStreamCaptureStatusNone) return MHD_OK;
    if ((rc = residual_report(A->d, rhs, x, J, st, hs))) return rc;
    if (st->nonfinite) {
        set_error("mhd_ens_solve: non-finite residual");
        return MHD_ENOCONV;
    }
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_spmm(mhd_shared A, const void* x, void* y, int J, int precision, mhd_stream_t s) try {
    CHECK_ARG(A && x && y, "mhd_ens_spmm: null argument");
    CHECK_ARG(x != y, "mhd_ens_spmm: x and y must not overlap");
    CHECK_ARG(precision == MHD_FP64 || precision == MHD_FP32_IR, "mhd_ens_spmm: bad precision");
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_spmm: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    CHECK_ARG(A->d.assembled, "mhd_ens_spmm: matrix not assembled");
    return spmm_shared(A->d, x, y, J, precision, as_stream(s));
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_timer_enable(int on) { return timer_enable(on); }
mhd_status mhd_ens_timer_op(int op) { return timer_op(op); }

mhd_status mhd_ens_timer_read(double* ms, int64_t* launches, double* nJ32, double* nJ64) try {
    return timer_read(ms, launches, nJ32, nJ64);
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_ctx_create(mhd_mesh m, const mhd_ctx_desc* d, mhd_ctx* out) try {
    CHECK_ARG(out, "mhd_ens_ctx_create: null output handle");
    *out = nullptr;
    CHECK_ARG(m && d, "mhd_ens_ctx_create: null argument");
    mhd_status rc = check_coeffs(&d->coeffs);
    if (rc) return rc;
    if ((rc = check_solver_opts(&d->solver))) return rc;
    CHECK_ARG(d->J_max >= 1 && d->J_max <= kMaxJ, "mhd_ens_ctx_create: J_max must be in [1, 4096]");
    CHECK_ARG(!d->graph || d->solver.fixed_cycles > 0,
              "mhd_ens_ctx_create: graph mode needs a fixed solver schedule (fixed_cycles > 0)");
    mhd_ctx c = new (std::nothrow) mhd_ctx_s;
    if (!c) return MHD_ENOMEM;
    c->mesh = m;
    c->desc = *d;
    auto fail = [&](mhd_status r) {
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->Av) mhd_ens_shared_free(c->Av);
        if (c->Aw) mhd_ens_shared_free(c->Aw);
        free_list(c->allocs);
        if (c->host_coef) (void)hipHostFree(c->host_coef);
        delete c;
        return r;
    };
    const bool compact = d->solver.fixed_cycles == 0;   // fixed schedules never compact
    if ((rc = shared_create(m, d->J_max, d->solver.restart, compact, &c->Av))) return fail(rc);
    if ((rc = shared_create(m, d->J_max, d->solver.restart, compact, &c->Aw))) return fail(rc);
    size_t blk = (size_t)m->d.n * d->J_max;
    if ((rc = dev_alloc(c->allocs, &c->bv, blk))) return fail(rc);
    if ((rc = dev_alloc(c->allocs, &c->bw, blk))) return fail(rc);
    if ((rc = dev_alloc(c->allocs, &c->Xv, blk))) return fail(rc);
    if ((rc = dev_alloc(c->allocs, &c->Xw, blk))) return fail(rc);
    if ((rc = dev_alloc(c->allocs, &c->coef, 2 * (size_t)d->J_max))) return fail(rc);
    if (d->solver.fixed_cycles > 0 && !d->serial) {
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
            set_error("mhd_ens_ctx_create: stream/event creation failed");
            return fail(MHD_EHIP);
        }
    }
    if ((rc = dev_alloc(c->allocs, &c->partial, (size_t)2048 * d->J_max + 1024))) return fail(rc);
    // tune (or take from the process-wide table) the node-row kernel plans for J_max
    // and build the data they use, so that no step allocates or synchronises for it
    if ((rc = autotune(c->Av->d, d->J_max, d->solver.precision, nullptr, false, nullptr))) return fail(rc);
    if ((rc = autotune(c->Aw->d, d->J_max, d->solver.precision, nullptr, false, nullptr))) return fail(rc);
    if (hipHostMalloc((void**)&c->host_coef, sizeof(double) * 2 * d->J_max, hipHostMallocDefault) != hipSuccess)
        return fail(MHD_ENOMEM);
    if (d->adjoint) {
        if (d->coeffs.convective != 0) {
            set_error("mhd_ens_ctx_create: the adjoint supports the skew-symmetric trilinear form only");
            return fail(MHD_EINVAL);
        }
        DevMesh& D = m->d;
        size_t vb = 2 * (size_t)D.nP2 * d->J_max;
        for (double** p : {&c->Tv, &c->Tv1, &c->Tw, &c->Tw1, &c->Kmv, &c->Kmw})
            if ((rc = dev_alloc(c->allocs, p, vb))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->tmeans, 8 * (size_t)D.nP2))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->eta_v, 14 * (size_t)D.n_el))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->eta_w, 14 * (size_t)D.n_el))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->js_v, 7 * (size_t)D.n_el))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->js_w, 7 * (size_t)D.n_el))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->Mf, 2 * (size_t)D.nP2))) return fail(rc);
        if ((rc = dev_alloc(c->allocs, &c->dots, 10 * (size_t)d->J_max))) return fail(rc);
    }
    *out = c;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_ctx_free(mhd_ctx c) try {
    if (!c) return MHD_OK;
    c->graph.reset();
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    mhd_ens_shared_free(c->Av);
    mhd_ens_shared_free(c->Aw);
    free_list(c->allocs);
    if (c->host_coef) (void)hipHostFree(c->host_coef);
    delete c;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_autotune(mhd_shared A, int J, int precision, mhd_tune_entry* out, int cap, int* count,
                            mhd_stream_t s) try {
    CHECK_ARG(A, "mhd_ens_autotune: null handle");
    CHECK_ARG(precision == MHD_FP64 || precision == MHD_FP32_IR, "mhd_ens_autotune: bad precision");
    CHECK_ARG(cap >= 0 && (cap == 0 || out), "mhd_ens_autotune: bad output array");
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_autotune: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    hipStream_t st = as_stream(s);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MHD_HIP(hipStreamIsCapturing(st, &cs));
    CHECK_ARG(cs == hipStreamCaptureStatusNone, "mhd_ens_autotune: stream is being captured");
    std::vector<mhd_tune_entry> rep;
    mhd_status rc = autotune(A->d, J, precision, st, true, &rep);
    if (rc) return rc;
    const int n = std::min<int>(cap, (int)rep.size());
    for (int i = 0; i < n; ++i) out[i] = rep[i];
    if (count) *count = n;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_set_plan(mhd_shared A, int J, int precision, int op, int vec, int group, int deep, int tile,
                            int waves) try {
    CHECK_ARG(A, "mhd_ens_set_plan: null handle");
    CHECK_ARG(precision == MHD_FP64 || precision == MHD_FP32_IR, "mhd_ens_set_plan: bad precision");
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_set_plan: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    return set_plan(A->d, J, precision, op, vec, group, deep, tile, waves);
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_get_plan(mhd_shared A, int J, int precision, int op, mhd_tune_entry* out) try {
    CHECK_ARG(A && out, "mhd_ens_get_plan: null argument");
    CHECK_ARG(precision == MHD_FP64 || precision == MHD_FP32_IR, "mhd_ens_get_plan: bad precision");
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_get_plan: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    return query_plan(A->d, J, precision, op, out);
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_prepare(mhd_shared A, int J, int precision, mhd_stream_t s) try {
    CHECK_ARG(A, "mhd_ens_prepare: null handle");
    CHECK_ARG(precision == MHD_FP64 || precision == MHD_FP32_IR, "mhd_ens_prepare: bad precision");
    if (J < 1 || J > A->d.Jmax) {
        set_error("mhd_ens_prepare: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    hipStream_t st = as_stream(s);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MHD_HIP(hipStreamIsCapturing(st, &cs));
    CHECK_ARG(cs == hipStreamCaptureStatusNone, "mhd_ens_prepare: stream is being captured");
    return autotune(A->d, J, precision, st, false, nullptr);
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_ctx_prepare(mhd_ctx ctx, int J, mhd_stream_t s) try {
    CHECK_ARG(ctx, "mhd_ens_ctx_prepare: null context");
    mhd_status rc = mhd_ens_prepare(ctx->Av, J, ctx->desc.solver.precision, s);
    if (rc == MHD_OK) rc = mhd_ens_prepare(ctx->Aw, J, ctx->desc.solver.precision, s);
    return rc;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_alloc_stats(int64_t* count, int64_t* bytes) try {
    if (count) *count = g_alloc_count.load();
    if (bytes) *bytes = g_alloc_bytes.load();
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_step(mhd_ctx ctx, double* V, double* W, double* Q, double* R, const mhd_step_inputs* in,
                        mhd_step_stats* st, mhd_stream_t s) try {
    CHECK_ARG(ctx && in, "mhd_ens_step: null argument");
    CHECK_ARG(V && W && Q && R, "mhd_ens_step: null state array");
    hipStream_t stv = as_stream(s);
    StepArgs a{V, W, Q, R, in->f1, in->f2, in->g_v, in->g_w, in->J};
    mhd_coeffs c;
    mhd_status rc = step_prepare(ctx, in, c, stv);
    if (rc) return rc;
    mhd_solve_stats sv{}, sw{};
    if (st && !ctx->desc.graph) {   // eager: the solves fill the caller's per-member arrays
        sv.relres = st->v.relres;
        sv.member_iters = st->v.member_iters;
        sw.relres = st->w.relres;
        sw.member_iters = st->w.member_iters;
    }
    mhd_status rs = MHD_OK;
    if (ctx->desc.graph) {
        CHECK_ARG(stv != nullptr, "mhd_ens_step: graph mode needs a non-null stream");
        if (!ctx->graph.valid || !(ctx->graph.key == a) || ctx->graph.stream != stv) {
            ctx->graph.reset();
            // kernel plans are fixed into the graph: those prepared at context
            // creation (or by mhd_ens_ctx_prepare for this J), else the defaults
            MHD_HIP(hipStreamBeginCapture(stv, hipStreamCaptureModeThreadLocal));
            rs = step_device(ctx, c, a, stv, &sv, &sw, true);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(stv, &graph);
            if (rs != MHD_OK && rs != MHD_ENOCONV) {
                if (graph) (void)hipGraphDestroy(graph);
                return rs;
            }
            if (e != hipSuccess) {
                set_error(std::string("mhd_ens_step: graph capture failed: ") + hipGetErrorString(e));
                return MHD_EHIP;
            }
            ctx->graph.graph = graph;
            MHD_HIP(hipGraphInstantiate(&ctx->graph.exec, graph, nullptr, nullptr, 0));
            ctx->graph.key = a;
            ctx->graph.stream = stv;
            ctx->graph.valid = true;
            ctx->graph.sv = sv;
            ctx->graph.sw = sw;
        }
        MHD_HIP(hipGraphLaunch(ctx->graph.exec, stv));
        sv = ctx->graph.sv;
        sw = ctx->graph.sw;
    } else {
        rs = step_device(ctx, c, a, stv, &sv, &sw, true);
        if (rs != MHD_OK && rs != MHD_ENOCONV) return rs;
    }
    if (st) {
        auto counts = [](mhd_solve_stats& d, const mhd_solve_stats& r) {
            d.min_block_rank = r.min_block_rank;
            d.iters = r.iters;
            d.cycles = r.cycles;
            d.max_relres = r.max_relres;
            d.converged = r.converged;
            d.nonfinite = r.nonfinite;
            d.norm_clamps = r.norm_clamps;
            d.compacted = r.compacted;
        };
        counts(st->v, sv);
        counts(st->w, sw);
        if (ctx->desc.solver.fixed_cycles > 0) {
            // a fixed schedule looks at no residual while it runs: report the final ones
            if ((rc = residual_report(ctx->Av->d, ctx->bv, ctx->Xv, a.J, &st->v, stv))) return rc;
            if ((rc = residual_report(ctx->Aw->d, ctx->bw, ctx->Xw, a.J, &st->w, stv))) return rc;
            for (mhd_solve_stats* q : {&st->v, &st->w})
                if (q->member_iters)
                    for (int j = 0; j < a.J; ++j) q->member_iters[j] = q->iters;
        }
        st->min_alpha = ctx->min_alpha;
        st->warnings = ctx->warnings | ((st->v.nonfinite || st->w.nonfinite) ? MHD_WARN_NONFINITE : 0);
        if ((rc = step_energy(ctx, a, stv, &st->energy))) return rc;
        if (st->warnings & MHD_WARN_NONFINITE) {
            set_error("mhd_ens_step: non-finite residual");
            return MHD_ENOCONV;
        }
    }
    if (rs == MHD_ENOCONV) {
        set_error("mhd_ens_step: a subproblem solve hit maxit");
        return MHD_ENOCONV;
    }
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_group_create(int n, const mhd_ctx* ctxs, mhd_group* out) try {
    CHECK_ARG(out, "mhd_ens_group_create: null output handle");
    *out = nullptr;
    CHECK_ARG(n >= 1 && n <= 64 && ctxs, "mhd_ens_group_create: need 1..64 contexts");
    for (int i = 0; i < n; ++i) {
        CHECK_ARG(ctxs[i], "mhd_ens_group_create: null context");
        CHECK_ARG(ctxs[i]->desc.solver.fixed_cycles > 0,
                  "mhd_ens_group_create: every context needs a fixed solver schedule (fixed_cycles > 0)");
    }
    mhd_group g = new (std::nothrow) mhd_group_s;
    if (!g) return MHD_ENOMEM;
    g->ctxs.assign(ctxs, ctxs + n);
    g->streams.resize(n, nullptr);
    g->done.resize(n, nullptr);
    for (int i = 0; i < n; ++i) {
        if (hipStreamCreateWithFlags(&g->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&g->done[i], hipEventDisableTiming) != hipSuccess) {
            mhd_ens_group_free(g);
            set_error("mhd_ens_group_create: stream/event creation failed");
            return MHD_EHIP;
        }
    }
    if (hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) != hipSuccess) {
        mhd_ens_group_free(g);
        set_error("mhd_ens_group_create: event creation failed");
        return MHD_EHIP;
    }
    *out = g;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_group_free(mhd_group g) try {
    if (!g) return MHD_OK;
    g->graph.reset();
    for (auto s : g->streams)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : g->done)
        if (e) (void)hipEventDestroy(e);
    if (g->fork) (void)hipEventDestroy(g->fork);
    delete g;
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_group_step(mhd_group g, double* const* V, double* const* W, double* const* Q, double* const* R,
                              const mhd_step_inputs* in, mhd_stream_t s) try {
    CHECK_ARG(g && V && W && Q && R && in, "mhd_ens_group_step: null argument");
    hipStream_t st = as_stream(s);
    CHECK_ARG(st != nullptr, "mhd_ens_group_step: needs a non-null stream (graph capture)");
    const int n = (int)g->ctxs.size();
    std::vector<StepArgs> args(n);
    std::vector<mhd_coeffs> cs(n);
    for (int i = 0; i < n; ++i) {
        CHECK_ARG(V[i] && W[i] && Q[i] && R[i], "mhd_ens_group_step: null state array");
        args[i] = StepArgs{V[i], W[i], Q[i], R[i], in[i].f1, in[i].f2, in[i].g_v, in[i].g_w, in[i].J};
        mhd_status rc = step_prepare(g->ctxs[i], &in[i], cs[i], st);
        if (rc) return rc;
    }
    // the mean viscosities, dt and mu enter the captured kernels by value: a change re-captures
    bool same = g->graph.valid && g->graph.stream == st && g->keys.size() == (size_t)n && g->coeffs.size() == (size_t)n;
    for (int i = 0; same && i < n; ++i)
        same = g->keys[i] == args[i] && g->coeffs[i].dt == cs[i].dt && g->coeffs[i].mu == cs[i].mu &&
               g->coeffs[i].nu_bar == cs[i].nu_bar && g->coeffs[i].num_bar == cs[i].num_bar;
    if (!same) {
        g->graph.reset();
        // kernel plans: those the contexts prepared (at creation for J_max), else the defaults
        MHD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        mhd_status rs = MHD_OK;
        hipError_t e = hipEventRecord(g->fork, st);
        for (int i = 0; i < n && rs == MHD_OK && e == hipSuccess; ++i) {
            e = hipStreamWaitEvent(g->streams[i], g->fork, 0);
            if (e != hipSuccess) break;
            mhd_solve_stats sv{}, sw{};
            // the ensembles of a group already run on parallel branches: no further split inside a branch
            rs = step_device(g->ctxs[i], cs[i], args[i], g->streams[i], &sv, &sw, false);
            if (rs == MHD_ENOCONV) rs = MHD_OK;
            if (rs == MHD_OK) e = hipEventRecord(g->done[i], g->streams[i]);
            if (rs == MHD_OK && e == hipSuccess) e = hipStreamWaitEvent(st, g->done[i], 0);
        }
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (rs != MHD_OK || e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (rs == MHD_OK) {
                set_error(std::string("mhd_ens_group_step: capture failed: ") +
                          hipGetErrorString(e != hipSuccess ? e : e2));
                return MHD_EHIP;
            }
            return rs;
        }
        g->graph.graph = graph;
        MHD_HIP(hipGraphInstantiate(&g->graph.exec, graph, nullptr, nullptr, 0));
        g->graph.stream = st;
        g->graph.valid = true;
        g->keys = args;
        g->coeffs = cs;
    }
    MHD_HIP(hipGraphLaunch(g->graph.exec, st));
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_adjoint_terminal(mhd_ctx ctx, const double* V, const double* W, double* lamV, double* lamW,
                                    int J, mhd_stream_t s) try {
    CHECK_ARG(ctx && V && W && lamV && lamW, "mhd_ens_adjoint_terminal: null argument");
    if (J < 1 || J > ctx->desc.J_max) {
        set_error("mhd_ens_adjoint_terminal: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    DevMesh& D = ctx->mesh->d;
    hipStream_t st = as_stream(s);
    double* zb = ctx->Av->d.zbar;
    hipError_t e = launch_mean(V, zb, 2 * (int64_t)D.nP2, J, st);
    if (e == hipSuccess) e = launch_energy_adjoint(D, zb, lamV, J, st);
    if (e == hipSuccess) e = launch_mean(W, zb, 2 * (int64_t)D.nP2, J, st);
    if (e == hipSuccess) e = launch_energy_adjoint(D, zb, lamW, J, st);
    if (e != hipSuccess) {
        set_error(std::string("mhd_ens_adjoint_terminal: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_adjoint_step(mhd_ctx ctx, const double* V_n, const double* W_n, const double* V_np1,
                                const double* W_np1, const double* lamV_np1, const double* lamW_np1,
                                double* lamV_n, double* lamW_n, const mhd_adjoint_inputs* in, double* grad,
                                mhd_step_stats* stt, mhd_stream_t s) try {
    CHECK_ARG(ctx && in, "mhd_ens_adjoint_step: null argument");
    CHECK_ARG(ctx->Tv, "mhd_ens_adjoint_step: context created without the adjoint workspace");
    CHECK_ARG(V_n && W_n && V_np1 && W_np1 && lamV_np1 && lamW_np1 && lamV_n && lamW_n,
              "mhd_ens_adjoint_step: null state array");
    CHECK_ARG(in->nu && in->nu_m, "mhd_ens_adjoint_step: null nu / nu_m");
    const int J = in->J;
    if (J < 1 || J > ctx->desc.J_max) {
        set_error("mhd_ens_adjoint_step: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    DevMesh& D = ctx->mesh->d;
    hipStream_t st = as_stream(s);
    double nub = 0, numb = 0;
    for (int j = 0; j < J; ++j) {
        nub += in->nu[j];
        numb += in->nu_m[j];
    }
    nub /= J;
    numb /= J;
    MHD_HIP(hipStreamSynchronize(st));   // the pinned staging buffer may still feed an earlier copy
    for (int j = 0; j < J; ++j) {
        ctx->host_coef[j] = 0.5 * (in->nu[j] - in->nu_m[j]);
        ctx->host_coef[J + j] = 0.5 * ((in->nu[j] - nub) + (in->nu_m[j] - numb));
    }
    MHD_HIP(hipMemcpyAsync(ctx->coef, ctx->host_coef, sizeof(double) * 2 * J, hipMemcpyHostToDevice, st));
    mhd_coeffs c = ctx->desc.coeffs;
    c.nu_bar = nub;
    c.num_bar = numb;
    DevShared& Av = ctx->Av->d;
    DevShared& Aw = ctx->Aw->d;
    mhd_status rc;
    if ((rc = assemble_shared_impl(D, c, W_n, J, Av, st))) return rc;    // zbar = <w>
    if ((rc = assemble_shared_impl(D, c, V_n, J, Aw, st))) return rc;    // zbar = <v>
    hipError_t e = launch_transpose_A(D, Av, st);
    if (e == hipSuccess) e = launch_transpose_A(D, Aw, st);
    if (e != hipSuccess) {
        set_error(std::string("mhd_ens_adjoint_step transpose: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    const size_t vel = sizeof(double) * 2 * (size_t)D.nP2 * J;
    const size_t prs = sizeof(double) * (size_t)D.nP1 * J;
    const int64_t poff = 2 * (int64_t)D.nP2 * J;
    MHD_HIP(hipMemcpyAsync(ctx->bv, lamV_np1, vel, hipMemcpyDeviceToDevice, st));
    MHD_HIP(hipMemcpyAsync(ctx->bw, lamW_np1, vel, hipMemcpyDeviceToDevice, st));
    MHD_HIP(hipMemsetAsync(ctx->bv + poff, 0, prs, st));
    MHD_HIP(hipMemsetAsync(ctx->bw + poff, 0, prs, st));
    MHD_HIP(hipMemsetAsync(ctx->Xv, 0, vel + prs, st));
    MHD_HIP(hipMemsetAsync(ctx->Xw, 0, vel + prs, st));
    mhd_solve_stats sv{}, sw{};
    if (stt) {   // the transposed solves fill the caller's per-member arrays
        sv.relres = stt->v.relres;
        sv.member_iters = stt->v.member_iters;
        sw.relres = stt->w.relres;
        sw.member_iters = stt->w.member_iters;
    }
    Av.transposed = Aw.transposed = true;
    mhd_status rv = solve_shared(Av, ctx->bv, ctx->Xv, J, ctx->desc.solver, &sv, st);
    mhd_status rw = (rv == MHD_OK || rv == MHD_ENOCONV) ? solve_shared(Aw, ctx->bw, ctx->Xw, J, ctx->desc.solver, &sw, st)
                                                        : rv;
    Av.transposed = Aw.transposed = false;
    if (rv != MHD_OK && rv != MHD_ENOCONV) return rv;
    if (rw != MHD_OK && rw != MHD_ENOCONV) return rw;
    const double* muv = ctx->Xv;
    const double* muw = ctx->Xw;
    const int64_t rows = 2 * (int64_t)D.nP2;
    double* Tvbar = ctx->tmeans;
    double* Tv1bar = ctx->tmeans + rows;
    double* Twbar = ctx->tmeans + 2 * rows;
    double* Tw1bar = ctx->tmeans + 3 * rows;
    const double eddy_c = 2.0 * c.mu * c.dt;
    e = launch_adj_T(D, muv, muw, V_n, W_n, V_np1, W_np1, ctx->Tv, ctx->Tv1, ctx->Tw, ctx->Tw1, J, st);
    if (e == hipSuccess) e = launch_mean(ctx->Tv, Tvbar, rows, J, st);
    if (e == hipSuccess) e = launch_mean(ctx->Tv1, Tv1bar, rows, J, st);
    if (e == hipSuccess) e = launch_mean(ctx->Tw, Twbar, rows, J, st);
    if (e == hipSuccess) e = launch_mean(ctx->Tw1, Tw1bar, rows, J, st);
    // eddy of S_w (l_v from V_n') against mu_w and W^{n+1}; eddy of S_v (l_w) against mu_v and V^{n+1}
    if (e == hipSuccess) e = launch_adj_eddy(D, V_n, Aw.zbar, muw, W_np1, ctx->eta_v, ctx->js_v, J, eddy_c, st);
    if (e == hipSuccess) e = launch_adj_eddy(D, W_n, Av.zbar, muv, V_np1, ctx->eta_w, ctx->js_w, J, eddy_c, st);
    if (e == hipSuccess)
        e = launch_adj_lambda(D, ctx->coef, muv, muw, V_n, W_n, Aw.zbar, Av.zbar, ctx->Tv, ctx->Tw, Tvbar, Tv1bar,
                              Twbar, Tw1bar, ctx->eta_v, ctx->js_v, ctx->eta_w, ctx->js_w, lamV_n, lamW_n, ctx->Kmv,
                              ctx->Kmw, J, c.dt, st);
    if (e == hipSuccess && grad) {
        int nt = 6;
        const double* X[8] = {ctx->Kmv, ctx->Kmv, ctx->Kmv, ctx->Kmw, ctx->Kmw, ctx->Kmw, muv, muw};
        const double* Y[8] = {W_n, V_n, V_np1, V_n, W_n, W_np1, ctx->Mf, ctx->Mf};
        int yv[8] = {0, 0, 0, 0, 0, 0, 1, 1};
        if (in->fhat) {
            e = launch_mass_vec_masked(D, in->fhat, ctx->Mf, st);
            nt = 8;
        } else {
            e = hipMemsetAsync(ctx->dots + 6 * J, 0, sizeof(double) * 2 * J, st);
        }
        if (e == hipSuccess) e = launch_multidot(X, Y, yv, nt, rows, J, ctx->partial, ctx->dots, st);
        if (e == hipSuccess) e = launch_adj_grad(ctx->dots, J, grad, st);
    }
    if (e != hipSuccess) {
        set_error(std::string("mhd_ens_adjoint_step: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    if (stt) {
        stt->v = sv;
        stt->w = sw;
        stt->energy = 0.0;
        stt->warnings = 0;
        stt->min_alpha = 0.0;
    }
    if (rv == MHD_ENOCONV || rw == MHD_ENOCONV) {
        set_error("mhd_ens_adjoint_step: a transposed solve hit maxit");
        return MHD_ENOCONV;
    }
    return MHD_OK;
} catch (...) {
    return exception_status();
}

mhd_status mhd_ens_adjoint_ic(mhd_ctx ctx, const double* lamV0, const double* lamW0, const double* modes, int nm,
                              double s_coupling, double* grad_ic, int J, mhd_stream_t s) try {
    CHECK_ARG(ctx && lamV0 && lamW0 && modes && grad_ic, "mhd_ens_adjoint_ic: null argument");
    CHECK_ARG(ctx->dots, "mhd_ens_adjoint_ic: context created without the adjoint workspace");
    CHECK_ARG(nm >= 1 && nm <= 4, "mhd_ens_adjoint_ic: nm must be in [1, 4]");
    CHECK_ARG(s_coupling >= 0 && std::isfinite(s_coupling), "mhd_ens_adjoint_ic: bad coupling number");
    if (J < 1 || J > ctx->desc.J_max) {
        set_error("mhd_ens_adjoint_ic: J outside [1, J_max]");
        return MHD_ESHAPE;
    }
    DevMesh& D = ctx->mesh->d;
    hipStream_t st = as_stream(s);
    const int64_t rows = 2 * (int64_t)D.nP2;
    const double* X[8];
    const double* Y[8];
    int yv[8];
    for (int m = 0; m < nm; ++m) {
        X[m] = lamV0;
        X[nm + m] = lamW0;
        Y[m] = Y[nm + m] = modes + (int64_t)m * rows;
        yv[m] = yv[nm + m] = 1;
    }
    hipError_t e = launch_multidot(X, Y, yv, 2 * nm, rows, J, ctx->partial, ctx->dots, st);
    if (e == hipSuccess) e = launch_ic_combine(ctx->dots, nm, J, std::sqrt(s_coupling), grad_ic, st);
    if (e != hipSuccess) {
        set_error(std::string("mhd_ens_adjoint_ic: ") + hipGetErrorString(e));
        return MHD_EHIP;
    }
    return MHD_OK;
} catch (...) {
    return exception_status();
}

}  // extern "C"
