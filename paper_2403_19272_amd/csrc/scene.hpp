// Internal scene state of the cloth library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cloth.h"

namespace cloth {

constexpr int TPB = 256;          // threads per block of the vertex/pair kernels
constexpr int MAX_OBST = 4;
constexpr double NO_HIT = 2.0;
constexpr int MAX_R = 192;        // widest basis: the packed FP64 Cholesky factor lives in LDS
constexpr int GRAM_CHUNKS = 512;
// A norm slot is DX_SUB sub-slots 64 bytes apart (DX_STRIDE u64 per slot):
// workgroup b folds its maximum into sub-slot b % DX_SUB, so that the
// atomics of a launch's workgroups do not queue on one address; the slot's
// value is the maximum over its sub-slots.
constexpr int DX_SUB = 16;
constexpr int DX_STRIDE = 8 * DX_SUB;  // contact-vertex chunks of the Gram partials
constexpr int RF_MAX = 64;        // residual-forwarding iterations per step at most
constexpr int CHEB_EST_SLOTS = 201;  // per-iteration norms of the Chebyshev estimate
constexpr int GRAM_GROUPS_MAX = 16;  // chunk groups of the first FP64 reduction level
constexpr int U_SEG = 32;         // local-step blocks summed per level-1 partial of U^T r0

// Step status bits (device word, 0 = the step succeeded).  The first four
// are the capacity overflows of the contact stages; a step that sets any of
// them, or a non-finite iterate, is rolled back to its starting state.
constexpr int STEP_OVF_QUERY = 1, STEP_OVF_CELL = 2, STEP_OVF_LIST = 4, STEP_OVF_CONS = 8;
constexpr int STEP_DIVERGED = 16;
constexpr int STEP_TANGLED = 32;
// Device counter words (ContactState::cnt, 32 ints).  The contact stages
// use [0..6], [9], [10], [12] (list counts), [16..24] (the time-of-impact
// chunk scheduler) and [25..26] (the heavy-query rescan); these are the
// step's: overflow bits of the running step, failure bits since the last
// stats read, the last step's status, the inner iterations and outer blocks
// the last step executed, and the tangle check's crossing and undecided
// counts ([28], [29]).
// [30] is set whenever a collision weight may have changed since the last
// factorization of the reduced matrix (a life span changed, a new
// constraint set, weights forced to k) and cleared by the factorization;
// [31] counts the factorizations since the last stats read.
constexpr int CNT_STEP_FAIL = 7, CNT_STICKY = 13, CNT_LAST_STATUS = 14, CNT_INNER_DONE = 15,
              CNT_OUTER_DONE = 27, CNT_TANGLES = 28, CNT_WCHG = 30, CNT_NFACT = 31;
constexpr int CNT_WORDS = 32;
static_assert(CNT_NFACT < CNT_WORDS, "counter words");

// LDS of the contact solve (factor and triangular solves in one workgroup):
// packed lower triangle, r inverse pivots and one zero entry
inline size_t chol_lds_bytes(int r) { return sizeof(double) * ((size_t)r * (r + 1) / 2 + r + 1); }

// Triangle record for the local step: corner ids, PD weight w = k_s * area,
// and the gradient rows g_j, g_k (g_i = -g_j - g_k) with F = sum_c x_c g_c^T.
struct TriRec {
    int v0, v1, v2;
    float w;
    float gj0, gj1, gk0, gk1;
};
static_assert(sizeof(TriRec) == 32, "TriRec layout");

// Analytic obstacle in the form the kernels read (FP64 so that the
// proximity decisions are taken in double precision).
struct ObstD {
    int kind;        // CLOTH_SPHERE / CLOTH_CYLINDER (axis a unit length)
    double c[3], a[3], R;
    double wh;       // spin about the axis times the time step (rad per step)
};

// Device pointers and sizes handed to kernels by value.
struct Dev {
    int nv, nt, ne, r;
    // SoA 3*nv arrays: [0,nv) x, [nv,2nv) y, [2nv,3nv) z
    float *x, *v, *xstar, *z, *xm, *xk, *xkm1, *xk1, *xt, *b, *WY;
    float4* x4;               // nv: AoS copy of x^k for the neighbour gathers
    float4* d4;               // nv: AoS delta = U q (gathered by the Jacobi sweep)
    float4* e4;               // nv: AoS first step of a rank-2 A-Jacobi iteration
    float* W;                 // nv: diagonal collision weights
    float* mh2;               // nv: m / h^2
    float* diag;              // nv: diag(H)
    const uint8_t* pinned;    // nv
    const int* rowptr;        // nv+1
    const int* col;           // nnz
    const float* val;         // nnz
    const int* sell_ptr;      // nv/64 slices + 1: SELL-64 off-diagonal part of H
    const int* sell_col;
    const float* sell_val;
    const TriRec* tri;        // nt
    const int* inc_ptr;       // nv+1: vertex -> (triangle << 2 | corner)
    const int* inc;           // 3*nt
    const int* edges;         // 2*ne (lexicographic, i < j)
    const void* U;            // nv*r, row-major, float or bf16 bits
    float* gpart;             // nblk * r * 3
    float* Qf;                // r * 3
    double* Qd;               // r * 3
    double* Ainv;             // r * r (no-contact inverse of Lambda~)
    double* Lam;              // r * r
    double* Amat;             // contact reduced matrix work: FP64 group sums of U^T W U
                              // (GRAM_GROUPS_MAX packed triangles), then A (one)
    double* cholf;            // the last factorization: packed L D L^T (r (r + 1) / 2) and 1 / D (r)
    double* gram_part;        // GRAM_CHUNKS * r * r Gram partials (FP64)
    unsigned long long* dxbits;  // per-iteration max |dx| as double bits
    double* gvec;             // r * 3: g = U^T r0 (FP64)
    float* UU;                // nv * r (r + 1) / 2: upper triangles of U_j U_j^T (Eq. (uu)), or null
    // contact (read when the contact flag is set)
    const int* vslot_ptr;     // nv+1: vertex -> slots of pair constraints
    const int* vslot;         // slot ids (4 * constraint + corner), sorted per vertex
    const float4* slot;       // per slot (w, w*y)
    int* ob_a;                // MAX_OBST * nv obstacle life spans (-1 = none)
    const ObstD* ob;          // obstacle table
    int nob;
    float kc, Kb;             // initial weight k and growth base K of Eq. (exp)
    double dhat;
    float smin, smax;         // strain limits of the projection (1, 1: rotation)
    float mu;                 // friction coefficient of obstacle contacts (0: none)
    double feps;              // sticking slip threshold eps_v h (m)
    // Tolerance mode: while `gate` is set and *gate != 0 the kernel returns
    // at once (the Jacobi sweep copies x^k forward instead), so a converged
    // loop runs its remaining launches of the fixed step graph as no-ops.
    const int* gate;
    int* fail;                // step status bits (non-finite iterates are flagged here)
};

struct Scene {
    // sizes and settings
    int nv = 0, nt = 0, ne = 0, nh = 0, r = 0;
    int64_t nnz = 0, nsell = 0;   // CSR nonzeros, SELL-64 entries
    double h = 0, density = 0, ks = 0, kb = 0, kc = 0, Kb = 2, dhat = 1e-3, alpha = 0.8;
    int amax = 20;
    int iters_in = 10, iters_out = 1, delay = 3, prec = CLOTH_PLAIN_FP32, self_contact = 0;
    double rho = 0, gamma = 0;
    double tol_in = 0, tol_out = 0;   // Algorithm 1 loop tolerances (<= 0: fixed budgets)
    double smin = 1, smax = 1;        // strain limits
    double mu = 0, feps = 0;          // obstacle friction coefficient, sticking slip eps_v h
    int debug_tangles = 0;            // check the end state of every step for intersecting triangles
    double bp_mu0 = 0.0, bp_kappa = 1.0;   // reusable candidate superset: box growth margins
    int bp_reuse = 0;                      // ... and whether it is used
    int r_warm = 0;                   // width of the modal warm-start basis (0: the reuse basis)
    int uu_store = 0;                 // contact matrix from the precomputed U_j U_j^T store
    int smoother = 0;                 // 0: Chebyshev-accelerated Jacobi, 1: rank-2 A-Jacobi
    int adapt_samples = 0;            // partial-CCD sample density from the change of rho*
    std::vector<int> perm;            // internal vertex i is the caller's perm[i] (empty: the caller's order)
    void* d_Uw = nullptr;             // its stored values (nv * r_warm)
    double* d_Ainvw = nullptr;        // inverse of its Galerkin matrix (r_warm * r_warm)
    bool warm_set = false;
    int64_t pair_cap = 0;
    bool basis_set = false;
    bool x4_valid = false;        // d.x4 holds x^k (written by the Jacobi sweep)
    int warm_iters = 0, rf_iters = 0;   // modal warm start / residual forwarding iterations
    double rf_toi = 0.5;                // forward when the exiting t_TOI is below this

    // host data (FP64 precompute)
    std::vector<int> tris, edges, hinges;  // hinges: 4 per interior edge
    std::vector<uint8_t> pinned;
    std::vector<double> rest, mass, area, g;  // g: 6 per triangle (g_i, g_j, g_k)
    std::vector<double> K, w_hinge;
    std::vector<int> rowptr, col;
    std::vector<double> val, diag;
    std::vector<int> sell_ptr, sell_col;   // off-diagonal SELL-64 copy of H (see host_build.cpp)
    std::vector<float> sell_val;
    std::vector<double> Ustored;   // nv*r stored-precision values as FP64
    std::vector<double> Lam;       // r*r
    std::vector<ObstD> obst;

    // device memory
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    bool arena_owned = false;
    Dev d{};
    int nblk = 0;                 // vertex blocks
    uint8_t* d_pinned = nullptr;
    float* d_rfdx = nullptr;      // forwarded residual dx (3*nv)
    int* d_gate = nullptr;        // [0] skip this inner iteration, [1] skip this outer block
    int nslots_cap = 0;           // entries of d.dxbits (norm slots)
    int *d_rowptr = nullptr, *d_col = nullptr, *d_inc_ptr = nullptr, *d_inc = nullptr,
        *d_edges = nullptr;
    float* d_val = nullptr;
    int *d_sell_ptr = nullptr, *d_sell_col = nullptr;
    float* d_sell_val = nullptr;
    TriRec* d_tri = nullptr;
    void* d_U = nullptr;
    double* d_dx_host_copy = nullptr;
    std::vector<float> omega;     // Chebyshev weights per inner index

    // stats of the last step
    cloth_step_stats last{};

    // whole-step graph: captured on a private stream, replayed on the caller's
    bool use_graph = true;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    float graph_g[3] = {0, 0, 0};

    // optional per-kernel timing: event pairs recorded around launches
    // second stream of the step (the contact matrix beside the local step),
    // joined by events; both are recorded into the step graph
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_used;   // (kernel id, pool index of the start event)
    std::vector<double> kt_ms;
    std::vector<int64_t> kt_n;
};

// kernel ids of the timing table
// (the outer CCD stage: K_BROAD broad phase other than the edge-edge
// counting pass K_QUERY_EE, K_TOI the time-of-impact kernel, K_OUTER the
// rest: set merge, obstacles, step length, compaction, filter, block set-up)
// (K_GRAM_CHOL: the contact matrix and its factorization, on the side
// stream beside the local step; K_CHOL_TRI: the solve on the factor)
enum KernelId {
    K_PREDICT = 0, K_LOCAL, K_REDUCE, K_EXPAND, K_JACOBI, K_TARGETS, K_GRAM_CHOL, K_PCCD, K_OUTER,
    K_BROAD, K_QUERY_EE, K_TOI, K_CHOL_TRI, K_MISC, K_COUNT
};
static const char* const kKernelNames[K_COUNT] = {
    "predict", "local_residual", "reduce_solve", "expand", "jacobi_cheb", "pair_targets",
    "gram_cholesky", "partial_ccd", "outer_set_filter", "broad_phase", "query_count_ee", "toi_merge",
    "contact_solve", "misc"};

// Timing brackets (api.cpp): no-ops unless the scene's timing is on.  For a
// single-kernel id (local residual, expand, Jacobi sweep, edge-edge query
// count, TOI) the next launch through launch_timed carries the events.
void timing_begin(Scene& s, int id, hipStream_t st);
void timing_end(Scene& s, hipStream_t st);

// host precompute (host_build.cpp)
std::vector<int> rcm_order(int nv, int nt, const int32_t* tris);
std::string build_scene(Scene& s, const cloth_mesh* mesh, const float* rest, double dt,
                        const cloth_material* mat, const cloth_solver_params* prm);
// device eigenbasis (eig.hip).  workspace: device memory of at least
// eig_workspace_bytes(nv, r) bytes, or null to allocate (and free) it here.
cloth_status device_eigenbasis(Scene& s, int r, int degree, int max_passes, double tol, std::vector<double>& U,
                               std::vector<double>& w, int* passes, double* max_res, std::string& err,
                               void* workspace);
// Bytes of workspace the device eigenbasis needs, and the size of the
// library's fixed per-GPU workspace array (eig_static_workspace).
constexpr size_t EIG_SCRATCH_BYTES = size_t(64) << 20;
size_t eig_workspace_bytes(int nv, int r);
// Device address of the current GPU's fixed workspace (EIG_SCRATCH_BYTES).
cloth_status eig_static_workspace(void** out, std::string& err);

}  // namespace cloth
