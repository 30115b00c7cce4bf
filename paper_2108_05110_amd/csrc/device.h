// Device-side data of libmhd_ens and launcher prototypes (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"

#define MHD_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::mhd::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
            return MHD_EHIP;                                                       \
        }                                                                          \
    } while (0)

namespace mhd {

constexpr int kMaxRestart = 40;    // Krylov basis length limit
constexpr int kMaxJ = 4096;        // member count limit of one handle

template <typename T>
struct DevCSR {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int max_row = 0;              // longest row
    int32_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;
};

struct DevLevel {
    int n = 0;
    double omega = kMgOmega;      // Jacobi damping of this level's sweeps
    DevCSR<double> L, P, R;
    DevCSR<double> Dn, Up;        // fused V-cycle halves (levels above the coarsest)
    double* dinv = nullptr;
    float* dinv32 = nullptr;
    double* cinv = nullptr;       // coarsest only, n x n
    float* cinv32 = nullptr;      // coarsest only, ld32 x ld32 with zeros past n
    int ld32 = 0;                 // n rounded up to a multiple of 16
};

// Device copy of a HostTiling (row tiles of the LDS-staged kernels)
struct DevTiling {
    int tx = 0, ty = 0, ntiles = 0, max_s2 = 0, max_s1 = 0, max_r2 = 0, max_r1 = 0;
    int32_t *r2_ptr = nullptr, *r2 = nullptr, *r2_self = nullptr;
    int32_t *r1_ptr = nullptr, *r1 = nullptr, *r1_self = nullptr;
    int32_t *s2_ptr = nullptr, *s2 = nullptr, *s1_ptr = nullptr, *s1 = nullptr;
    int32_t *a_loc = nullptr, *bt_loc = nullptr, *b_loc = nullptr;
    int32_t *ta_rp = nullptr, *ta_loc = nullptr, *ta_gp = nullptr;
    int32_t *tbt_rp = nullptr, *tbt_loc = nullptr, *tbt_gp = nullptr;
    int32_t *tb_rp = nullptr, *tb_loc = nullptr, *tb_gp = nullptr;
    int max_ea = 0, max_ebt = 0, max_eb = 0;
};
constexpr int kTileShapes = 3;          // square tiles of 8, 12 or 16 half-steps
inline int tile_edge(int id) { return id == 1 ? 8 : id == 2 ? 12 : 16; }

// Row-per-lane tiles on the device (layout as HostEll).  Entries are packed
// with their LDS offset: B^T and B entries (mesh constants) as (offset, first
// value, second value, 0) in bm; A entries as (offset, value) in an array of
// each shared operator (DevShared::ellA), copied from am0 (values 0) and given
// its values by the assembly through posA (CSR position of an A entry -> its
// entry index).
struct DevEll {
    int tx = 0, ty = 0, m = 0, ntiles = 0, max_lds = 0, max_lds1 = 0, max_lds2 = 0, max_blocks = 0, max_blocks2 = 0;
    int max_k = 0;
    int64_t nent = 0;
    int32_t *tile = nullptr, *s2 = nullptr, *s1 = nullptr, *blk = nullptr, *rows = nullptr, *self = nullptr;
    int4* bm = nullptr;
    int2* am0 = nullptr;
    int32_t* posA = nullptr;
};
// shapes 1-3: rectangles of 16 x 16, 32 x 8 and 16 x 8 half-steps with 16
// members per workgroup; 4-6: the same with 8 members
constexpr int kEllShapes = 6;
inline int ell_tx(int id) { return (id - 1) % 3 == 1 ? 32 : 16; }
inline int ell_ty(int id) { return (id - 1) % 3 == 0 ? 16 : 8; }
inline int ell_m(int id) { return id > 3 ? 8 : 16; }
constexpr double kJacobiOmega = 0.6;   // velocity-block Jacobi damping when the options leave it 0
struct DevMesh {
    HostMesh host;
    int nP2 = 0, nP1 = 0, n_el = 0, n_dir = 0, pin = -1;
    int64_t n = 0;
    double* xy = nullptr;
    double* geo = nullptr;        // n_el x 6: detJ, Jinv[2][2], pad
    int32_t* tri = nullptr;       // n_el x 6
    int32_t* tri1 = nullptr;      // n_el x 3
    uint8_t* dir = nullptr;       // nP2
    int32_t* dir_index = nullptr; // nP2: position in dir_nodes or -1
    int32_t* dir_nodes = nullptr;
    int32_t* hs_p2 = nullptr;     // (2 ny + 1) x (2 nx + 1): half-step grid point -> P2 id or -1
    int32_t* cell_el = nullptr;   // ny x nx: cell -> lower element (upper = +1) or -1
    int32_t* p1_of_p2 = nullptr;  // nP2: P1 id of a vertex node, -1 for an edge node
    int nx = 0, ny = 0;           // cell grid
    int32_t *A_rowptr = nullptr, *A_col = nullptr, *A_row = nullptr;
    int32_t *Bt_rowptr = nullptr, *Bt_col = nullptr;
    int32_t *B_rowptr = nullptr, *B_col = nullptr;
    int64_t nnzA = 0, nnzBt = 0, nnzB = 0;
    int max_row = 0;              // longest row of the A, B^T and B patterns
    int max_row_bt = 0;           // longest row of the B^T pattern
    int32_t *gA_ptr = nullptr, *gA_idx = nullptr;
    int32_t *gB_ptr = nullptr, *gB_idx = nullptr;
    int32_t *gBt_ptr = nullptr, *gBt_idx = nullptr;
    int32_t *inc_ptr = nullptr, *inc = nullptr;
    double *valM = nullptr, *valK = nullptr;      // scalar P2 mass / stiffness
    double *valB = nullptr, *valBt = nullptr;     // 2 values per entry, BC rows applied
    float *valB32 = nullptr, *valBt32 = nullptr;
    double* diagp = nullptr;
    float* diagp32 = nullptr;
    // transposed operator: slot permutations and the constant transposed divergence blocks
    int32_t* permA = nullptr;                     // nnz_A: slot (i,k) -> slot (k,i)
    int32_t* permBtB = nullptr;                   // nnz_Bt: B^T slot (i,m) -> B slot (m,i)
    double *valB_T = nullptr, *valBt_T = nullptr; // B pattern / B^T pattern, 2 values per entry
    float *valB_T32 = nullptr, *valBt_T32 = nullptr;
    double* mp = nullptr;                         // lumped P1 mass
    double* mp_inv = nullptr;
    uint8_t* pfix = nullptr;                      // nP1: fixed rows of the pressure Laplacian
    std::vector<DevLevel> levels;
    double levels_dt = -1.0, levels_nuc = -1.0;   // the (dt, nu_c) the levels' values were built for
    DevTiling* tiling[kTileShapes + 1] = {};   // by shape id 1..kTileShapes, built on demand
    DevEll* ell[kEllShapes + 1] = {};          // row-per-lane tiles by shape id 1..kEllShapes, built on demand
    int32_t* pair_sched[9] = {};               // paired-row SpMM wave order by units per wavefront (4, 8)
    // small scratch for the stand-alone RHS call (member coefficients, means)
    double* scratch_coef = nullptr;               // 2 * kMaxJ
    double* scratch_mean = nullptr;               // 2 nP2
    std::vector<void*> allocs;
};

// Scott-Vogelius meshes (Alfeld refinement) have no half-step grid: the kernels
// built on it (row tiles, the strip right-hand side) are replaced by CSR-only
// and node-gather kernels there
inline bool sv_mesh(const DevMesh& m) { return m.host.desc.element == MHD_ELEMENT_SCOTT_VOGELIUS; }

struct GmresWork {
    int restart = 0;
    int64_t nrows = 0;
    int Jmax = 0;
    void* basis = nullptr;        // (restart+1) blocks of nrows*Jmax (sized for double)
    void* zbuf = nullptr;         // preconditioned vector
    void* wbuf = nullptr;         // product / work
    void* tbuf = nullptr;         // velocity right-hand side inside the preconditioner
    void* z2buf = nullptr;        // Jacobi ping-pong
    double* r64 = nullptr;        // fp64 residual (n x J)
    double* cb = nullptr;         // compacted right-hand sides and iterates of the members still
    double* cx = nullptr;         // unconverged (n x Jmax each; adaptive handles only)
    int32_t* cidx = nullptr;      // their member indices (Jmax)
    double* H = nullptr;          // (restart+1) x restart x J
    double* cs = nullptr;         // restart x J
    double* sn = nullptr;
    double* g = nullptr;          // (restart+1) x J
    double* y = nullptr;          // restart x J
    double* beta = nullptr;       // J
    double* bnorm = nullptr;      // J
    double* hcol = nullptr;       // (restart+1) x J current column
    double* res = nullptr;        // J residual estimates
    double* partial = nullptr;    // reduction partials
    int64_t partial_len = 0;
    int nblk_cap = 512;           // blocks of the column-reduction kernels for this J_max
    double* host_res = nullptr;   // pinned host copy (J)
    std::vector<void*> mg_x, mg_x2, mg_b, mg_r;   // per level (n_l x Jmax, sized for double)
    void* mg_y0 = nullptr;        // finest level: the first V-cycle's result when two are run
    void* dense_part = nullptr;   // partial products of the coarsest dense solve (kDenseKS x n_c x Jmax)
    void** dptrs = nullptr;       // device array of the basis block pointers
    double* bmat = nullptr;       // 2 Jmax^2: J x J matrices of the block solver (Jmax <= kBlockMaxJ)
    void* zbasis = nullptr;       // restart FP32 blocks: the preconditioned basis vectors of FP32 solves
    void** zptrs = nullptr;       // device array of their pointers
};

struct DevShared {
    DevMesh* mesh = nullptr;
    int Jmax = 0;
    double* valA = nullptr;       // nnzA
    float* valA32 = nullptr;
    double* valA_T = nullptr;     // transposed values (adjoint solves)
    float* valA_T32 = nullptr;
    bool transposed = false;      // solver uses the transposed operator
    double* dinvA = nullptr;      // nP2 inverse diagonal of A
    float* dinvA32 = nullptr;
    double* zbar = nullptr;       // 2 nP2
    double* l2 = nullptr;         // n_el x 7
    double* elem = nullptr;       // n_el x 36
    mhd_coeffs coeffs{};
    bool assembled = false;
    int2* ellA[kEllShapes + 1] = {};    // packed A entries of the row-per-lane tiles (FP32 values)
    bool ell_live[kEllShapes + 1] = {};  // a plan uses the tiling: assemblies refresh ellA
    GmresWork gw;
    // this handle's values of the pressure Schur-approximation hierarchy (patterns
    // shared with the mesh's levels), for its own (dt, nu_c)
    std::vector<DevLevel> levels;
    double schur_dt = -1.0, schur_nuc = -1.0;
    std::vector<void*> allocs;
};
constexpr int kBlockMaxJ = 128;   // block GMRES: J in {16, 32, 64, 128}

// Every device allocation of the library goes through dev_malloc, which counts
// them (count and bytes since load) for mhd_ens_alloc_stats.
hipError_t dev_malloc(void** p, size_t bytes);

// ---------------------------------------------------------------- launchers (assemble.hip)
void upload_ref_tables(const RefTables& t);
hipError_t launch_const_assembly(DevMesh& m, double* elembuf, hipStream_t s);
hipError_t launch_mean(const double* z, double* zbar, int64_t rows, int J, hipStream_t s);
hipError_t launch_eddy_l2(const DevMesh& m, const double* z, const double* zbar, double* l2, int J,
                          hipStream_t s);
hipError_t launch_assemble_A(const DevMesh& m, const mhd_coeffs& c, const double* zbar, const double* l2,
                             double* elem, double* valA, float* valA32, double* dinvA, float* dinvA32,
                             hipStream_t s);
hipError_t launch_member_coefs(const double* nu, const double* nu_m, int J, double* coef, hipStream_t s);
// right-hand sides of one subproblem in one pass, FP64 or (precision MHD_FP32_IR)
// FP32 output; every row of rhs (n x J) is written
hipError_t launch_rhs_strip(const DevMesh& m, const mhd_coeffs& c, int J, const double* self_n, const double* other_n,
                            const double* obar, const double* coef, const double* forcing, const double* bc,
                            void* rhs, int precision, hipStream_t s);
hipError_t launch_energy_partial(const DevMesh& m, const double* vbar, double* out, hipStream_t s);

// ---------------------------------------------------------------- solver (solve.hip)
mhd_status alloc_gmres(DevShared& S, int restart, bool compact);
mhd_status solve_shared(DevShared& S, const double* rhs, double* x, int J, const mhd_solver_opts& o,
                        mhd_solve_stats* st, hipStream_t s);
mhd_status spmm_shared(DevShared& S, const void* x, void* y, int J, int precision, hipStream_t s);
mhd_status residual_report(DevShared& S, const double* b, const double* x, int J, mhd_solve_stats* out,
                           hipStream_t st);
mhd_status autotune(DevShared& S, int J, int precision, hipStream_t st, bool force,
                    std::vector<mhd_tune_entry>* report);
mhd_status set_plan(DevShared& S, int J, int precision, int op, int vec, int group, int deep, int tile, int waves);
mhd_status query_plan(DevShared& S, int J, int precision, int op, mhd_tune_entry* out);
mhd_status timer_op(int op);
mhd_status timer_enable(int on);
mhd_status timer_read(double* ms, int64_t* launches, double* nJ32, double* nJ64);
mhd_status saddle_residual64(DevShared& S, const double* b, const double* x, double* r, int J, hipStream_t s);
// copies the FP32 A values into every row-per-lane entry array the operator holds
hipError_t scatter_ell_values(DevShared& S, hipStream_t s);

hipError_t launch_reduce_rows(const double* partial, int nblk, int64_t width, double* out, hipStream_t s);

// ---------------------------------------------------------------- adjoint (adjoint.hip)
void upload_ref_tables_adjoint(const RefTables& t);
hipError_t launch_transpose_const(DevMesh& m, hipStream_t s);
hipError_t launch_transpose_A(DevMesh& m, DevShared& S, hipStream_t s);
hipError_t launch_energy_adjoint(const DevMesh& m, const double* zbar, double* lam, int J, hipStream_t s);
hipError_t launch_mass_vec_masked(const DevMesh& m, const double* f, double* out, hipStream_t s);
hipError_t launch_adj_T(const DevMesh& m, const double* muv, const double* muw, const double* V, const double* W,
                        const double* V1, const double* W1, double* Tv, double* Tv1, double* Tw, double* Tw1, int J,
                        hipStream_t s);
hipError_t launch_adj_eddy(const DevMesh& m, const double* Z, const double* zbar, const double* mu, const double* X,
                           double* eta, int32_t* jstar, int J, double eddy_c, hipStream_t s);
hipError_t launch_adj_lambda(const DevMesh& m, const double* coef, const double* muv, const double* muw, const double* V,
                             const double* W, const double* vbar, const double* wbar, const double* Tv,
                             const double* Tw, const double* Tvbar, const double* Tv1bar, const double* Twbar,
                             const double* Tw1bar, const double* eta_v, const int32_t* js_v, const double* eta_w,
                             const int32_t* js_w, double* lamV, double* lamW, double* Kmv, double* Kmw, int J,
                             double dt, hipStream_t s);
hipError_t launch_multidot(const double* const* X, const double* const* Y, const int* yvec, int nt, int64_t R, int J,
                           double* partial, double* out, hipStream_t s);
hipError_t launch_adj_grad(const double* d, int J, double* grad, hipStream_t s);
hipError_t launch_ic_combine(const double* d, int nm, int J, double sq, double* grad_ic, hipStream_t s);

// pressure post-processing: p -= (sum_k m_k p_k) / sum_k m_k per member
hipError_t launch_pressure_zero_mean(const DevMesh& m, double* p, int J, double* partial, hipStream_t s);

}  // namespace mhd
