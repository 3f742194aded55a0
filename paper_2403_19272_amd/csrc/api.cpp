// C ABI of the cloth library: scene lifetime, state I/O, the time step and
// the stage-level entry points.  Host code only enqueues device work; the
// numerics live in pd_kernels.hip and contact_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <new>
#include <string>
#include <vector>

#include "contact.hpp"
#include "kernels.hpp"
#include "scene.hpp"

using namespace cloth;

namespace {

thread_local std::string g_err;

cloth_status fail(cloth_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHECK(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(CLOTH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

template <typename T>
T* carve(Scene& s, size_t count) {
    size_t bytes = (sizeof(T) * count + 255) & ~(size_t)255;
    if (s.arena_used + bytes > s.arena_bytes) return nullptr;
    T* p = reinterpret_cast<T*>(s.arena + s.arena_used);
    s.arena_used += bytes;
    return p;
}

uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

float bf16_to_f(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// AoS (x0,y0,z0,...) host <-> SoA device planes; with a vertex order, row
// perm[i] of the caller's array is internal vertex i
void aos_to_soa(const float* a, std::vector<float>& s, int n, const std::vector<int>& perm = {}) {
    s.resize(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const size_t src = perm.empty() ? i : perm[i];
        for (int c = 0; c < 3; ++c) s[(size_t)c * n + i] = a[3 * src + c];
    }
}
void soa_to_aos(const std::vector<float>& s, float* a, int n, const std::vector<int>& perm = {}) {
    for (int i = 0; i < n; ++i) {
        const size_t dst = perm.empty() ? i : perm[i];
        for (int c = 0; c < 3; ++c) a[3 * dst + c] = s[(size_t)c * n + i];
    }
}
// rows of an n x r basis between the caller's order and the internal one
static std::vector<double> rows_to_internal(const double* U, int n, int r, const std::vector<int>& perm) {
    std::vector<double> out((size_t)n * r);
    for (int i = 0; i < n; ++i) std::copy(U + (size_t)perm[i] * r, U + (size_t)(perm[i] + 1) * r, &out[(size_t)i * r]);
    return out;
}
static void rows_to_caller(const std::vector<double>& Ui, double* U, int n, int r, const std::vector<int>& perm) {
    for (int i = 0; i < n; ++i)
        std::copy(&Ui[(size_t)i * r], &Ui[(size_t)(i + 1) * r], U + (size_t)(perm.empty() ? i : perm[i]) * r);
}
static bool reordered(const Scene& s) { return !s.perm.empty(); }

// Symmetric positive definite inverse by Cholesky (FP64, host).
bool spd_inverse(const std::vector<double>& A, int r, std::vector<double>& inv) {
    std::vector<double> L(A);
    for (int k = 0; k < r; ++k) {
        double dkk = L[(size_t)k * r + k];
        for (int j = 0; j < k; ++j) dkk -= L[(size_t)k * r + j] * L[(size_t)k * r + j];
        if (!(dkk > 0)) return false;
        dkk = std::sqrt(dkk);
        L[(size_t)k * r + k] = dkk;
        for (int i = k + 1; i < r; ++i) {
            double a = L[(size_t)i * r + k];
            for (int j = 0; j < k; ++j) a -= L[(size_t)i * r + j] * L[(size_t)k * r + j];
            L[(size_t)i * r + k] = a / dkk;
        }
    }
    inv.assign((size_t)r * r, 0.0);
    std::vector<double> y(r);
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < r; ++i) {
            double a = (i == c) ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) a -= L[(size_t)i * r + j] * y[j];
            y[i] = a / L[(size_t)i * r + i];
        }
        for (int i = r - 1; i >= 0; --i) {
            double a = y[i];
            for (int j = i + 1; j < r; ++j) a -= L[(size_t)j * r + i] * inv[(size_t)j * r + c];
            inv[(size_t)i * r + c] = a / L[(size_t)i * r + i];
        }
    }
    return true;
}

std::vector<float> cheb_weights(int n, double rho, int delay) {
    std::vector<float> w(std::max(n, 1));
    double prev = 1.0;
    for (int k = 0; k < (int)w.size(); ++k) {
        double om;
        if (k < delay)
            om = 1.0;
        else if (k == delay)
            om = 2.0 / (2.0 - rho * rho);
        else
            om = 4.0 / (4.0 - rho * rho * prev);
        prev = om;
        w[k] = (float)om;
    }
    return w;
}

struct Rot {
    float* p[3];
};

template <typename T>
T* cv(const Carver& f, size_t count) {
    return static_cast<T*>(f(sizeof(T) * count));
}

// Norm slots of d.dxbits: one per inner iteration of the step (block-major),
// then the residual-forwarding iterations, then one per outer block (the
// change of x over the block); at least the Chebyshev estimate's.
int slot_inner(const Scene& s, int o, int k) { return o * s.iters_in + k; }
int slot_rf(const Scene& s, int k) { return s.iters_out * s.iters_in + k; }
int slot_outer(const Scene& s, int o) { return s.iters_out * s.iters_in + RF_MAX + o; }
int slots_needed(const Scene& s) { return std::max(slot_outer(s, s.iters_out), CHEB_EST_SLOTS); }
// the device address of norm slot i (DX_SUB sub-slots, see scene.hpp)
unsigned long long* dx_slot(Scene& s, int i) { return s.d.dxbits + (size_t)i * DX_STRIDE; }
// the values of the first n norm slots (the maximum over each slot's
// sub-slots), read after the work on st
std::vector<unsigned long long> read_slots(Scene& s, int n, hipStream_t st) {
    std::vector<unsigned long long> raw((size_t)n * DX_STRIDE), out(n, 0ull);
    if (hipMemcpyAsync(raw.data(), s.d.dxbits, 8 * raw.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return out;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < DX_SUB; ++k) out[i] = std::max(out[i], raw[(size_t)i * DX_STRIDE + 8 * k]);
    return out;
}

}  // namespace

// Carves every device buffer of a scene from `carve` (the arena, or a
// counting carver for the footprint query).
static cloth_status layout_scene(Scene& s, ContactState& c, const Carver& carve_fn) {
    const int n = s.nv;
    Dev& d = s.d;
    d.nv = n;
    d.nt = s.nt;
    d.ne = s.ne;
    d.r = s.r;
    s.nblk = (n + TPB - 1) / TPB;
    float** vecs[] = {&d.x, &d.v, &d.xstar, &d.z, &d.xm, &d.xk, &d.xkm1, &d.xk1, &d.xt, &d.b, &d.WY};
    for (float** pv : vecs) {
        *pv = cv<float>(carve_fn, 3 * (size_t)n);
        if (!*pv) return fail(CLOTH_E_OOM, "arena exhausted (state)");
    }
    d.x4 = cv<float4>(carve_fn, n);
    d.d4 = cv<float4>(carve_fn, n);
    d.e4 = cv<float4>(carve_fn, n);
    d.W = cv<float>(carve_fn, n);
    d.mh2 = cv<float>(carve_fn, n);
    d.diag = cv<float>(carve_fn, n);
    s.d_pinned = cv<uint8_t>(carve_fn, n);
    s.d_rowptr = cv<int>(carve_fn, n + 1);
    s.d_col = cv<int>(carve_fn, (size_t)s.nnz);
    s.d_val = cv<float>(carve_fn, (size_t)s.nnz);
    const int nsl = (n + 63) / 64;
    const size_t nsell = (size_t)s.nsell;
    s.d_sell_ptr = cv<int>(carve_fn, nsl + 1);
    s.d_sell_col = cv<int>(carve_fn, nsell + 1);
    s.d_sell_val = cv<float>(carve_fn, nsell + 1);
    s.d_tri = cv<TriRec>(carve_fn, s.nt);
    s.d_inc_ptr = cv<int>(carve_fn, n + 1);
    s.d_inc = cv<int>(carve_fn, 3 * (size_t)s.nt);
    s.d_edges = cv<int>(carve_fn, 2 * (size_t)s.ne);
    size_t ubytes = (s.prec == CLOTH_MIXED ? 2 : 4) * (size_t)n * s.r;
    s.d_U = cv<char>(carve_fn, ubytes);
    // the warm-start basis (optional) and the work buffers of the wider basis
    const int rw = std::max(s.r, s.r_warm);
    if (s.r_warm > 0) {
        s.d_Uw = cv<char>(carve_fn, (s.prec == CLOTH_MIXED ? 2 : 4) * (size_t)n * s.r_warm);
        s.d_Ainvw = cv<double>(carve_fn, (size_t)s.r_warm * s.r_warm);
        if (!s.d_Uw || !s.d_Ainvw) return fail(CLOTH_E_OOM, "arena exhausted (warm basis)");
    }
    d.gpart = cv<float>(carve_fn, (size_t)s.nblk * rw * 3);
    d.Qf = cv<float>(carve_fn, (size_t)rw * 3);
    d.Qd = cv<double>(carve_fn, (size_t)rw * 3);
    d.Ainv = cv<double>(carve_fn, (size_t)s.r * s.r);
    d.Lam = cv<double>(carve_fn, (size_t)s.r * s.r);
    d.Amat = cv<double>(carve_fn, (size_t)(GRAM_GROUPS_MAX + 1) * s.r * (s.r + 1) / 2);
    d.gram_part = cv<double>(carve_fn, (size_t)GRAM_CHUNKS * s.r * s.r);
    d.cholf = cv<double>(carve_fn, (size_t)s.r * (s.r + 1) / 2 + s.r);
    d.UU = nullptr;
    if (s.uu_store) {
        d.UU = cv<float>(carve_fn, (size_t)n * s.r * (s.r + 1) / 2);
        if (!d.UU) return fail(CLOTH_E_OOM, "arena exhausted (U_j U_j^T store)");
    }
    s.nslots_cap = slots_needed(s);
    d.dxbits = cv<unsigned long long>(carve_fn, (size_t)s.nslots_cap * DX_STRIDE);
    s.d_rfdx = cv<float>(carve_fn, 3 * (size_t)n);
    s.d_gate = cv<int>(carve_fn, 4);
    if (!d.x4 || !d.d4 || !d.W || !d.mh2 || !d.diag || !s.d_pinned || !s.d_rowptr || !s.d_col || !s.d_val || !s.d_tri ||
        !s.d_sell_ptr || !s.d_sell_col || !s.d_sell_val ||
        !s.d_inc_ptr || !s.d_inc || !s.d_edges || !s.d_U || !d.gpart || !d.Qf || !d.Qd || !d.Ainv ||
        !d.Lam || !d.Amat || !d.gram_part || !d.cholf || !d.dxbits || !s.d_rfdx || !s.d_gate)
        return fail(CLOTH_E_OOM, "arena exhausted");
    return contact_layout(s, c, carve_fn);
}

static size_t dry_footprint(const Scene& src) {
    Scene s;
    s.nv = src.nv;
    s.nt = src.nt;
    s.ne = src.ne;
    s.nnz = src.nnz;
    s.nsell = src.nsell;
    s.r = src.r;
    s.r_warm = src.r_warm;
    s.bp_reuse = src.bp_reuse;
    s.uu_store = src.uu_store;
    s.smoother = src.smoother;
    s.iters_in = src.iters_in;
    s.iters_out = src.iters_out;
    s.prec = src.prec;
    s.self_contact = src.self_contact;
    s.pair_cap = src.pair_cap;
    s.nblk = src.nblk;
    ContactState c;
    size_t used = 0;
    Carver count = [&](size_t bytes) -> void* {
        used += (bytes + 255) & ~(size_t)255;
        return reinterpret_cast<void*>(used);  // never dereferenced
    };
    layout_scene(s, c, count);
    return used + 4096;
}

// ------------------------------------------------------------------ timing

namespace cloth {

// Timing pairs: the single-kernel operations (local residual, expand,
// Jacobi sweep) get the kernel's own start/end time (the launcher passes the
// events to hipExtLaunchKernelGGL); the other operations, which may launch
// several kernels, are bracketed by two recorded events.
static bool single_kernel_op(int id) {
    return id == K_LOCAL || id == K_EXPAND || id == K_JACOBI || id == K_QUERY_EE || id == K_TOI;
}

static void t_begin(Scene& s, int id, hipStream_t st) {
    if (!s.timing) return;
    size_t k = s.ev_used.size() * 2;
    while (s.ev_pool.size() < k + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            s.timing = false;
            return;
        }
        s.ev_pool.push_back(e);
    }
    if (single_kernel_op(id))
        set_kernel_events(s.ev_pool[k], s.ev_pool[k + 1]);
    else
        (void)hipEventRecord(s.ev_pool[k], st);
    s.ev_used.push_back({id, (int)k});
}

static void t_end(Scene& s, hipStream_t st) {
    if (!s.timing || s.ev_used.empty()) return;
    if (single_kernel_op(s.ev_used.back().first))
        clear_kernel_events();
    else
        (void)hipEventRecord(s.ev_pool[s.ev_used.back().second + 1], st);
}

// folds the recorded pairs into the per-kernel totals (after a sync)
static void t_collect(Scene& s) {
    if (s.kt_ms.size() != K_COUNT) {
        s.kt_ms.assign(K_COUNT, 0.0);
        s.kt_n.assign(K_COUNT, 0);
    }
    for (auto& u : s.ev_used) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s.ev_pool[u.second], s.ev_pool[u.second + 1]) == hipSuccess) {
            s.kt_ms[u.first] += ms;
            s.kt_n[u.first] += 1;
        }
    }
    s.ev_used.clear();
}

void timing_begin(Scene& s, int id, hipStream_t st) { t_begin(s, id, st); }
void timing_end(Scene& s, hipStream_t st) { t_end(s, st); }

#define TIMED(id, expr)            \
    do {                           \
        t_begin(s, id, st);        \
        auto rc_t_ = (expr);       \
        t_end(s, st);              \
        if (rc_t_ != decltype(rc_t_)(0)) return fail_any(rc_t_, #expr); \
    } while (0)

static cloth_status fail_any(hipError_t e, const char* what) {
    return fail(CLOTH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
static cloth_status fail_any(cloth_status c, const char*) { return c; }

// One inner iteration on the device state: x^k = d.xk, x^{k-1} = d.xkm1 ->
// d.xk1; then buffers rotate so that d.xk holds x^{k+1}.
static cloth_status inner_iteration(cloth_scene_s* sc, int k, int slot, hipStream_t st, bool linear,
                                    float omega_override, bool force_k = false, int prev_slot = -1,
                                    bool targets_ready = false) {
    Scene& s = sc->s;
    ContactState& c = sc->c;
    Dev& d = s.d;
    int has_contact = (c.active && !linear) ? 1 : 0;
    if (k == 0 || !s.x4_valid) TIMED(K_MISC, launch_aos4(d.xk, d.x4, s.nv, st));
    if (has_contact) {
        // (the previous iteration's partial CCD may have written them already)
        if (!targets_ready) TIMED(K_TARGETS, contact_prepare_iteration(s, c, force_k, st));
        // fork: the contact matrix needs only the collision weights, fixed
        // once the targets are; it is formed and factored on the side stream
        // while the local step and U^T r0 run
        HIPCHECK(hipEventRecord(s.ev_fork, st));
        HIPCHECK(hipStreamWaitEvent(s.side, s.ev_fork, 0));
        {
            hipStream_t st_main = st;
            st = s.side;
            TIMED(K_GRAM_CHOL, contact_factor(s, c, force_k, st));
            st = st_main;
        }
        HIPCHECK(hipEventRecord(s.ev_join, s.side));
    }
    TIMED(K_LOCAL, launch_local_residual(d, s.prec, has_contact | (linear ? 2 : 0) | (force_k ? 4 : 0), st));
    TIMED(K_REDUCE, launch_reduce_solve(d, s.nblk, has_contact, c.gpart2, st));
    if (has_contact) {
        HIPCHECK(hipStreamWaitEvent(st, s.ev_join, 0));   // join
        TIMED(K_CHOL_TRI, contact_solve(s, c, st));
    }
    TIMED(K_EXPAND, launch_expand(d, s.prec, 0, st));
    float om = omega_override > 0 ? omega_override : s.omega[std::min(k, (int)s.omega.size() - 1)];
    if (s.smoother == 1 && !linear) {
        // rank-2 A-Jacobi: two damped Jacobi steps, no Chebyshev blend
        TIMED(K_JACOBI, launch_jacobi_cheb(d, 1.0f, (float)s.gamma, has_contact, dx_slot(s, slot),
                                           prev_slot >= 0 ? dx_slot(s, prev_slot) : nullptr, st, 1));
        TIMED(K_JACOBI, launch_jacobi_cheb(d, 1.0f, (float)s.gamma, has_contact, dx_slot(s, slot),
                                           prev_slot >= 0 ? dx_slot(s, prev_slot) : nullptr, st, 2));
    } else {
        TIMED(K_JACOBI, launch_jacobi_cheb(d, om, (float)s.gamma, has_contact, dx_slot(s, slot),
                                           prev_slot >= 0 ? dx_slot(s, prev_slot) : nullptr, st));
    }
    float* t = d.xkm1;
    d.xkm1 = d.xk;
    d.xk = d.xk1;
    d.xk1 = t;
    s.x4_valid = true;   // the sweep wrote x^{k+1} to d.x4 as well
    return CLOTH_OK;
}

// One modal warm-start iteration on d.xk (collisions ignored): local step,
// q = Lambda~^{-1} U^T (b - H x), x <- x + U q (Algorithm 1, before the
// first full CCD).
static cloth_status modal_iteration(cloth_scene_s* sc, hipStream_t st) {
    Scene& s = sc->s;
    ContactState& c = sc->c;
    // the warm-start basis when one is set (its own width and inverse
    // Galerkin matrix; the work buffers are sized for the wider basis)
    Dev d = s.d;
    if (s.warm_set) {
        d.U = s.d_Uw;
        d.r = s.r_warm;
        d.Ainv = s.d_Ainvw;
    }
    TIMED(K_MISC, launch_aos4(d.xk, d.x4, s.nv, st));
    TIMED(K_LOCAL, launch_local_residual(d, s.prec, 0, st));
    TIMED(K_REDUCE, launch_reduce_solve(d, s.nblk, 0, c.gpart2, st));
    TIMED(K_EXPAND, launch_expand(d, s.prec, 1, st));
    float* t = s.d.xk;
    s.d.xk = s.d.xt;
    s.d.xt = t;
    s.x4_valid = false;
    return CLOTH_OK;
}

}  // namespace cloth

// ------------------------------------------------------------------ ABI

extern "C" {

const char* cloth_status_string(cloth_status s) {
    switch (s) {
        case CLOTH_OK: return "ok";
        case CLOTH_E_INVALID: return "invalid argument";
        case CLOTH_E_MESH: return "invalid mesh";
        case CLOTH_E_OOM: return "out of device memory";
        case CLOTH_E_CAPACITY: return "buffer capacity exceeded";
        case CLOTH_E_DIVERGED: return "diverged";
        case CLOTH_E_TANGLED: return "tangled";
        case CLOTH_E_DEVICE: return "device error";
        default: return "unknown status";
    }
}

const char* cloth_last_error(void) { return g_err.c_str(); }

cloth_status cloth_vertex_order(const cloth_mesh* mesh, int32_t* order) {
    if (!mesh || !mesh->tris || !order || mesh->nv <= 0 || mesh->nt <= 0) return fail(CLOTH_E_INVALID, "null argument");
    for (size_t i = 0; i < 3 * (size_t)mesh->nt; ++i)
        if (mesh->tris[i] < 0 || mesh->tris[i] >= mesh->nv) return fail(CLOTH_E_MESH, "triangle index out of range");
    std::vector<int> o = rcm_order(mesh->nv, mesh->nt, mesh->tris);
    std::copy(o.begin(), o.end(), order);
    return CLOTH_OK;
}

cloth_status cloth_query_footprint(const cloth_mesh* mesh, const cloth_solver_params* params, size_t* bytes) {
    if (!mesh || !params || !bytes) return fail(CLOTH_E_INVALID, "null argument");
    if (!mesh->tris || mesh->nv <= 0 || mesh->nt <= 0) return fail(CLOTH_E_INVALID, "empty mesh");
    // count the nonzero pattern (diagonal + triangle corners + hinge
    // stencils) from the connectivity alone
    std::vector<std::vector<int>> nb(mesh->nv);
    std::vector<std::pair<int, int>> ed;
    std::vector<std::vector<int>> opp;
    {
        std::vector<std::pair<std::pair<int, int>, int>> e3;
        for (int t = 0; t < mesh->nt; ++t)
            for (int c = 0; c < 3; ++c) {
                int a = mesh->tris[3 * t + c], b = mesh->tris[3 * t + (c + 1) % 3],
                    o = mesh->tris[3 * t + (c + 2) % 3];
                if (a < 0 || a >= mesh->nv || b < 0 || b >= mesh->nv || o < 0 || o >= mesh->nv)
                    return fail(CLOTH_E_MESH, "triangle index out of range");
                e3.push_back({{std::min(a, b), std::max(a, b)}, o});
                nb[a].push_back(b);
                nb[a].push_back(o);
            }
        std::sort(e3.begin(), e3.end());
        for (size_t i = 0; i < e3.size();) {
            size_t j = i;
            while (j < e3.size() && e3[j].first == e3[i].first) ++j;
            ed.push_back(e3[i].first);
            if (j - i == 2) {
                int v[4] = {e3[i].first.first, e3[i].first.second, e3[i].second, e3[i + 1].second};
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b)
                        if (a != b) nb[v[a]].push_back(v[b]);
            }
            i = j;
        }
    }
    int64_t nnz = 0, nsell = 0;
    int slice_w = 0;
    for (int v = 0; v < mesh->nv; ++v) {
        auto& l = nb[v];
        l.push_back(v);
        std::sort(l.begin(), l.end());
        int len = (int)(std::unique(l.begin(), l.end()) - l.begin());
        nnz += len;
        slice_w = std::max(slice_w, len - 1);
        if (v % 64 == 63 || v == mesh->nv - 1) {
            nsell += 64 * (int64_t)slice_w;
            slice_w = 0;
        }
    }
    Scene ds;
    ds.nv = mesh->nv;
    ds.nt = mesh->nt;
    ds.ne = (int)ed.size();
    ds.nnz = nnz;
    ds.nsell = nsell;
    ds.r = params->r;
    ds.r_warm = params->r_warm;
    ds.uu_store = params->uu_store ? 1 : 0;
    ds.smoother = params->smoother;
    ds.bp_reuse = params->broad_reuse ? 1 : 0;
    ds.iters_in = std::max(1, params->iters_inner);
    ds.iters_out = std::max(1, params->iters_outer);
    ds.prec = params->precision;
    ds.self_contact = params->self_contact;
    ds.pair_cap = params->pair_capacity > 0 ? params->pair_capacity : (int64_t)128 * mesh->nv;
    ds.nblk = (ds.nv + TPB - 1) / TPB;
    *bytes = dry_footprint(ds);
    return CLOTH_OK;
}

cloth_status cloth_init(const cloth_mesh* mesh, const float* rest_xyz, const cloth_material* mat, double dt,
                        const cloth_solver_params* params, void* dev_arena, size_t arena_bytes,
                        cloth_scene* out) {
    if (!mesh || !rest_xyz || !mat || !params || !out) return fail(CLOTH_E_INVALID, "null argument");
    if (params->r < 8 || params->r > MAX_R || params->r % 8 != 0)
        return fail(CLOTH_E_INVALID, "r must be a multiple of 8 in [8, " + std::to_string(MAX_R) + "]");
    if (params->iters_inner <= 0 || params->iters_outer <= 0)
        return fail(CLOTH_E_INVALID, "iteration budgets must be positive");
    if (params->r_warm != 0 && (params->r_warm < 8 || params->r_warm > MAX_R || params->r_warm % 8 != 0))
        return fail(CLOTH_E_INVALID, "r_warm must be 0 or a multiple of 8 in [8, " + std::to_string(MAX_R) + "]");
    if (params->debug_tangles && !params->self_contact)
        return fail(CLOTH_E_INVALID, "the tangle check needs self contact on");
    if ((int64_t)params->iters_inner * params->iters_outer > 65536)
        return fail(CLOTH_E_INVALID, "iters_inner * iters_outer must be at most 65536");
    if (!std::isfinite(params->tol_inner) || !std::isfinite(params->tol_outer))
        return fail(CLOTH_E_INVALID, "tolerances must be finite");
    {
        const bool unset = mat->sigma_min == 0 && mat->sigma_max == 0;
        if (!unset && !(mat->sigma_min > 0 && mat->sigma_min <= 1.0 && mat->sigma_max >= 1.0 &&
                        std::isfinite(mat->sigma_max)))
            return fail(CLOTH_E_INVALID, "strain limits must satisfy 0 < sigma_min <= 1 <= sigma_max");
    }
    if (params->precision != CLOTH_PLAIN_FP32 && params->precision != CLOTH_MIXED)
        return fail(CLOTH_E_INVALID, "unknown precision");
    if (params->smoother != 0 && params->smoother != 1) return fail(CLOTH_E_INVALID, "unknown smoother");
    if (!(mat->friction >= 0 && std::isfinite(mat->friction)) || !std::isfinite(mat->friction_eps_v))
        return fail(CLOTH_E_INVALID, "friction must be finite and >= 0");
    std::unique_ptr<cloth_scene_s> sc(new (std::nothrow) cloth_scene_s());
    if (!sc) return fail(CLOTH_E_OOM, "host allocation");
    Scene& s = sc->s;
    // optional vertex reorder: the scene is built on the renumbered mesh
    // (triangles sorted by their lowest new vertex), and every host array
    // that crosses the boundary is mapped between the two orders
    cloth_mesh pm = *mesh;
    std::vector<int32_t> ptris;
    std::vector<uint8_t> ppin;
    std::vector<float> prest;
    if (params->reorder) {
        for (size_t i = 0; i < 3 * (size_t)mesh->nt; ++i)
            if (mesh->tris[i] < 0 || mesh->tris[i] >= mesh->nv) return fail(CLOTH_E_MESH, "triangle index out of range");
        s.perm = rcm_order(mesh->nv, mesh->nt, mesh->tris);
        std::vector<int> inv(mesh->nv);
        for (int i = 0; i < mesh->nv; ++i) inv[s.perm[i]] = i;
        std::vector<int> tord(mesh->nt);
        std::iota(tord.begin(), tord.end(), 0);
        auto lo = [&](int t) {
            return std::min({inv[mesh->tris[3 * t]], inv[mesh->tris[3 * t + 1]], inv[mesh->tris[3 * t + 2]]});
        };
        std::stable_sort(tord.begin(), tord.end(), [&](int a, int b) { return lo(a) < lo(b); });
        ptris.resize(3 * (size_t)mesh->nt);
        for (int t = 0; t < mesh->nt; ++t)
            for (int c = 0; c < 3; ++c) ptris[3 * (size_t)t + c] = inv[mesh->tris[3 * (size_t)tord[t] + c]];
        prest.resize(3 * (size_t)mesh->nv);
        for (int i = 0; i < mesh->nv; ++i)
            for (int c = 0; c < 3; ++c) prest[3 * (size_t)i + c] = rest_xyz[3 * (size_t)s.perm[i] + c];
        if (mesh->pinned) {
            ppin.resize(mesh->nv);
            for (int i = 0; i < mesh->nv; ++i) ppin[i] = mesh->pinned[s.perm[i]];
            pm.pinned = ppin.data();
        }
        pm.tris = ptris.data();
        rest_xyz = prest.data();
    }
    std::string err = build_scene(s, &pm, rest_xyz, dt, mat, params);
    if (!err.empty()) return fail(CLOTH_E_MESH, err);
    s.nblk = (s.nv + TPB - 1) / TPB;
    size_t need = dry_footprint(s);
    if (dev_arena) {
        if (arena_bytes < need)
            return fail(CLOTH_E_OOM, "arena of " + std::to_string(arena_bytes) + " bytes, need " +
                                         std::to_string(need));
        s.arena = static_cast<char*>(dev_arena);
        s.arena_bytes = arena_bytes;
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) return fail(CLOTH_E_OOM, "hipMalloc of the scene arena");
        s.arena = static_cast<char*>(p);
        s.arena_bytes = need;
        s.arena_owned = true;
    }
    cloth_status lrc = layout_scene(s, sc->c, [&](size_t bytes) -> void* { return carve<char>(s, bytes); });
    if (lrc != CLOTH_OK) return lrc;
    const int n = s.nv;
    Dev& d = s.d;
    d.pinned = s.d_pinned;
    d.rowptr = s.d_rowptr;
    d.col = s.d_col;
    d.val = s.d_val;
    d.sell_ptr = s.d_sell_ptr;
    d.sell_col = s.d_sell_col;
    d.sell_val = s.d_sell_val;
    d.tri = s.d_tri;
    d.inc_ptr = s.d_inc_ptr;
    d.inc = s.d_inc;
    d.edges = s.d_edges;
    d.U = s.d_U;
    d.smin = (float)s.smin;
    d.mu = (float)s.mu;
    d.feps = s.feps;
    d.smax = (float)s.smax;

    // static uploads
    std::vector<float> tmp(3 * (size_t)n);
    std::vector<float> f(n);
    for (int v = 0; v < n; ++v) f[v] = (float)(s.mass[v] / (dt * dt));
    HIPCHECK(hipMemcpy(d.mh2, f.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    for (int v = 0; v < n; ++v) f[v] = (float)s.diag[v];
    HIPCHECK(hipMemcpy(d.diag, f.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(s.d_pinned, s.pinned.data(), n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(s.d_rowptr, s.rowptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(s.d_col, s.col.data(), sizeof(int) * s.nnz, hipMemcpyHostToDevice));
    {
        std::vector<float> vf(s.val.begin(), s.val.end());
        HIPCHECK(hipMemcpy(s.d_val, vf.data(), sizeof(float) * s.nnz, hipMemcpyHostToDevice));
    }
    HIPCHECK(hipMemcpy(s.d_sell_ptr, s.sell_ptr.data(), sizeof(int) * s.sell_ptr.size(), hipMemcpyHostToDevice));
    if (!s.sell_col.empty()) {
        HIPCHECK(hipMemcpy(s.d_sell_col, s.sell_col.data(), sizeof(int) * s.sell_col.size(), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s.d_sell_val, s.sell_val.data(), sizeof(float) * s.sell_val.size(),
                           hipMemcpyHostToDevice));
    }
    {
        std::vector<TriRec> tr(s.nt);
        for (int t = 0; t < s.nt; ++t) {
            const double* g = &s.g[6 * (size_t)t];
            tr[t] = {s.tris[3 * t], s.tris[3 * t + 1], s.tris[3 * t + 2], (float)(s.ks * s.area[t]),
                     (float)g[2], (float)g[3], (float)g[4], (float)g[5]};
        }
        HIPCHECK(hipMemcpy(s.d_tri, tr.data(), sizeof(TriRec) * s.nt, hipMemcpyHostToDevice));
        std::vector<int> cnt(n + 1, 0), inc(3 * (size_t)s.nt);
        for (int t = 0; t < s.nt; ++t)
            for (int c = 0; c < 3; ++c) cnt[s.tris[3 * t + c] + 1]++;
        for (int v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int t = 0; t < s.nt; ++t)
            for (int c = 0; c < 3; ++c) inc[fill[s.tris[3 * t + c]]++] = (t << 2) | c;
        HIPCHECK(hipMemcpy(s.d_inc_ptr, cnt.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(s.d_inc, inc.data(), sizeof(int) * 3 * s.nt, hipMemcpyHostToDevice));
    }
    HIPCHECK(hipMemcpy(s.d_edges, s.edges.data(), sizeof(int) * 2 * s.ne, hipMemcpyHostToDevice));
    // initial state: rest at rest
    for (int v = 0; v < n; ++v)
        for (int c = 0; c < 3; ++c) tmp[(size_t)c * n + v] = rest_xyz[3 * (size_t)v + c];
    HIPCHECK(hipMemcpy(d.x, tmp.data(), sizeof(float) * 3 * n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemset(d.v, 0, sizeof(float) * 3 * n));
    HIPCHECK(hipMemset(d.W, 0, sizeof(float) * n));
    HIPCHECK(hipMemset(d.WY, 0, sizeof(float) * 3 * n));
    HIPCHECK(hipMemset(s.d_rfdx, 0, sizeof(float) * 3 * n));
    cloth_status rc = contact_upload(s, sc->c);
    if (rc != CLOTH_OK) return rc;
    // the step's second stream (default priority) and its fork / join events
    HIPCHECK(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming));
    HIPCHECK(hipDeviceSynchronize());
    *out = sc.release();
    return CLOTH_OK;
}

cloth_status cloth_system_matrix(cloth_scene sc, int64_t* nnz, int32_t* row_ptr, int32_t* col, double* val) {
    if (!sc || !nnz) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    *nnz = s.nnz;
    if (!reordered(s)) {
        if (row_ptr) std::copy(s.rowptr.begin(), s.rowptr.end(), row_ptr);
        if (col) std::copy(s.col.begin(), s.col.end(), col);
        if (val) std::copy(s.val.begin(), s.val.end(), val);
        return CLOTH_OK;
    }
    // rows and columns back in the caller's order, columns sorted per row
    const int n = s.nv;
    std::vector<int32_t> rp(n + 1, 0);
    for (int i = 0; i < n; ++i) rp[s.perm[i] + 1] = s.rowptr[i + 1] - s.rowptr[i];
    for (int i = 0; i < n; ++i) rp[i + 1] += rp[i];
    if (row_ptr) std::copy(rp.begin(), rp.end(), row_ptr);
    if (col || val) {
        std::vector<std::pair<int, double>> row;
        for (int i = 0; i < n; ++i) {
            row.clear();
            for (int k = s.rowptr[i]; k < s.rowptr[i + 1]; ++k) row.push_back({s.perm[s.col[k]], s.val[k]});
            std::sort(row.begin(), row.end());
            int32_t o = rp[s.perm[i]];
            for (auto& e : row) {
                if (col) col[o] = e.first;
                if (val) val[o] = e.second;
                ++o;
            }
        }
    }
    return CLOTH_OK;
}

cloth_status cloth_estimate_chebyshev(cloth_scene sc, void* stream);

// The recorded step graph holds the scene's settings as kernel arguments
// (Chebyshev weights, obstacle count, step options); a setter that changes
// them drops it so that the next step records it again.
static cloth_status drop_graph(Scene& s) {
    if (s.graph_exec) {
        HIPCHECK(hipGraphExecDestroy(s.graph_exec));
        s.graph_exec = nullptr;
    }
    return CLOTH_OK;
}

}  // extern "C"
namespace cloth {
cloth_status scene_drop_graph(cloth_scene_s* sc) { return drop_graph(sc->s); }
}  // namespace cloth
extern "C" {

// Rounds a basis U (nv x r FP64, row-major; pinned rows stored as zero) to
// the storage precision into dst, keeps the stored values, and forms
// L = U~^T H U~ in FP64 (symmetrised) and its inverse.
static cloth_status store_basis(Scene& s, const double* U, int r, void* dst, std::vector<double>& Ustored,
                                std::vector<double>& Lam, std::vector<double>& inv) {
    const int n = s.nv;
    Ustored.assign((size_t)n * r, 0.0);
    std::vector<float> uf;
    std::vector<uint16_t> ub;
    if (s.prec == CLOTH_MIXED)
        ub.assign((size_t)n * r, 0);
    else
        uf.assign((size_t)n * r, 0.f);
    for (int v = 0; v < n; ++v) {
        if (s.pinned[v]) continue;
        for (int c = 0; c < r; ++c) {
            size_t i = (size_t)v * r + c;
            float f = (float)U[i];
            if (s.prec == CLOTH_MIXED) {
                ub[i] = to_bf16(f);
                Ustored[i] = bf16_to_f(ub[i]);
            } else {
                uf[i] = f;
                Ustored[i] = f;
            }
        }
    }
    std::vector<double> HU((size_t)n * r, 0.0);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < n; ++v) {
        double* out = &HU[(size_t)v * r];
        for (int j = s.rowptr[v]; j < s.rowptr[v + 1]; ++j) {
            double a = s.val[j];
            const double* u = &Ustored[(size_t)s.col[j] * r];
            for (int c = 0; c < r; ++c) out[c] += a * u[c];
        }
    }
    Lam.assign((size_t)r * r, 0.0);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < r; ++a)
        for (int v = 0; v < n; ++v) {
            double ua = Ustored[(size_t)v * r + a];
            if (ua == 0.0) continue;
            const double* h = &HU[(size_t)v * r];
            double* row = &Lam[(size_t)a * r];
            for (int b = 0; b < r; ++b) row[b] += ua * h[b];
        }
    for (int a = 0; a < r; ++a)
        for (int b = a + 1; b < r; ++b) {
            double m = 0.5 * (Lam[(size_t)a * r + b] + Lam[(size_t)b * r + a]);
            Lam[(size_t)a * r + b] = Lam[(size_t)b * r + a] = m;
        }
    if (!spd_inverse(Lam, r, inv)) return fail(CLOTH_E_INVALID, "U~^T H U~ is not positive definite");
    if (s.prec == CLOTH_MIXED)
        HIPCHECK(hipMemcpy(dst, ub.data(), ub.size() * 2, hipMemcpyHostToDevice));
    else
        HIPCHECK(hipMemcpy(dst, uf.data(), uf.size() * 4, hipMemcpyHostToDevice));
    return CLOTH_OK;
}

static cloth_status set_basis_internal(cloth_scene sc, const double* U, int32_t r);

cloth_status cloth_set_basis(cloth_scene sc, const double* U, int32_t r) {
    if (!sc || !U) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    if (r != s.r) return fail(CLOTH_E_INVALID, "basis width differs from params.r");
    if (!reordered(s)) return set_basis_internal(sc, U, r);
    std::vector<double> Ui = rows_to_internal(U, s.nv, r, s.perm);
    return set_basis_internal(sc, Ui.data(), r);
}

// U in the internal vertex order
static cloth_status set_basis_internal(cloth_scene sc, const double* U, int32_t r) {
    Scene& s = sc->s;
    if (drop_graph(s) != CLOTH_OK) return CLOTH_E_DEVICE;
    if (r != s.r) return fail(CLOTH_E_INVALID, "basis width differs from params.r");
    std::vector<double> inv;
    cloth_status rc0 = store_basis(s, U, r, s.d_U, s.Ustored, s.Lam, inv);
    if (rc0 != CLOTH_OK) return rc0;
    HIPCHECK(hipMemcpy(s.d.Ainv, inv.data(), sizeof(double) * r * r, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(s.d.Lam, s.Lam.data(), sizeof(double) * r * r, hipMemcpyHostToDevice));
    if (s.uu_store) {
        cloth_status rc = contact_build_uu(s);
        if (rc != CLOTH_OK) return rc;
    }
    s.basis_set = true;
    if (s.rho <= 0 || s.gamma <= 0) {
        cloth_status rc = cloth_estimate_chebyshev(sc, nullptr);
        if (rc != CLOTH_OK) return rc;
    }
    s.omega = cheb_weights(std::max(s.iters_in, s.rf_iters), s.rho, s.delay);
    return CLOTH_OK;
}

cloth_status cloth_set_warm_basis(cloth_scene sc, const double* U, int32_t r_warm) {
    if (!sc || !U) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    if (s.r_warm <= 0) return fail(CLOTH_E_INVALID, "the scene was created without a warm-start basis (r_warm)");
    if (r_warm != s.r_warm) return fail(CLOTH_E_INVALID, "basis width differs from params.r_warm");
    if (drop_graph(s) != CLOTH_OK) return CLOTH_E_DEVICE;
    std::vector<double> stored, lam, inv;
    std::vector<double> Ui;
    if (reordered(s)) {
        Ui = rows_to_internal(U, s.nv, r_warm, s.perm);
        U = Ui.data();
    }
    cloth_status rc = store_basis(s, U, r_warm, s.d_Uw, stored, lam, inv);
    if (rc != CLOTH_OK) return rc;
    HIPCHECK(hipMemcpy(s.d_Ainvw, inv.data(), sizeof(double) * r_warm * r_warm, hipMemcpyHostToDevice));
    s.warm_set = true;
    return CLOTH_OK;
}

cloth_status cloth_set_step_options(cloth_scene sc, int32_t warm_iters, int32_t rf_iters, double rf_toi) {
    if (!sc || warm_iters < 0 || rf_iters < 0) return fail(CLOTH_E_INVALID, "bad step options");
    if (rf_iters > RF_MAX)
        return fail(CLOTH_E_INVALID, "rf_iters must be at most " + std::to_string(RF_MAX));
    Scene& s = sc->s;
    s.warm_iters = warm_iters;
    s.rf_iters = rf_iters;
    s.rf_toi = rf_toi;
    if (s.basis_set) s.omega = cheb_weights(std::max(s.iters_in, s.rf_iters), s.rho, s.delay);
    return drop_graph(s);
}

cloth_status cloth_get_forwarded(cloth_scene sc, float* dx) {
    if (!sc || !dx) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    std::vector<float> t(3 * (size_t)s.nv);
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(t.data(), s.d_rfdx, 12 * (size_t)s.nv, hipMemcpyDeviceToHost));
    soa_to_aos(t, dx, s.nv, s.perm);
    return CLOTH_OK;
}

cloth_status cloth_compute_basis(cloth_scene sc, int32_t r, int32_t degree, int32_t max_passes, double tol,
                                 double* U, double* ritz, int32_t* passes, double* residual) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    if (r != s.r) return fail(CLOTH_E_INVALID, "basis width differs from params.r");
    if (degree < 1 || max_passes < 1) return fail(CLOTH_E_INVALID, "degree and passes must be positive");
    std::vector<double> Uh, w;
    std::string err;
    int p = 0;
    double res = 0;
    cloth_status rc = device_eigenbasis(s, r, degree, max_passes, tol, Uh, w, &p, &res, err, nullptr);
    if (rc != CLOTH_OK) return fail(rc, err);
    if (U) rows_to_caller(Uh, U, s.nv, r, s.perm);
    if (ritz) std::copy(w.begin(), w.end(), ritz);
    if (passes) *passes = p;
    if (residual) *residual = res;
    return set_basis_internal(sc, Uh.data(), r);
}

cloth_status cloth_compute_basis_static(cloth_scene sc, int32_t r, int32_t degree, int32_t max_passes, double tol,
                                        double* U, double* ritz, int32_t* passes, double* residual) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    if (r != s.r) return fail(CLOTH_E_INVALID, "basis width differs from params.r");
    if (degree < 1 || max_passes < 1) return fail(CLOTH_E_INVALID, "degree and passes must be positive");
    const size_t need = eig_workspace_bytes(s.nv, r);
    if (need > EIG_SCRATCH_BYTES)
        return fail(CLOTH_E_INVALID, "the basis iteration needs " + std::to_string(need) +
                                         " bytes of workspace; the fixed workspace holds " +
                                         std::to_string(EIG_SCRATCH_BYTES) + " (use cloth_compute_basis)");
    std::string err;
    void* ws = nullptr;
    cloth_status rc = eig_static_workspace(&ws, err);
    if (rc != CLOTH_OK) return fail(rc, err);
    std::vector<double> Uh, w;
    int p = 0;
    double res = 0;
    rc = device_eigenbasis(s, r, degree, max_passes, tol, Uh, w, &p, &res, err, ws);
    if (rc != CLOTH_OK) return fail(rc, err);
    if (U) rows_to_caller(Uh, U, s.nv, r, s.perm);
    if (ritz) std::copy(w.begin(), w.end(), ritz);
    if (passes) *passes = p;
    if (residual) *residual = res;
    return set_basis_internal(sc, Uh.data(), r);
}

cloth_status cloth_add_obstacle(cloth_scene sc, const cloth_obstacle* ob) {
    if (!sc || !ob) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    if ((int)s.obst.size() >= MAX_OBST) return fail(CLOTH_E_INVALID, "too many obstacles");
    if (ob->kind != CLOTH_SPHERE && ob->kind != CLOTH_CYLINDER) return fail(CLOTH_E_INVALID, "obstacle kind");
    if (!(ob->radius > 0)) return fail(CLOTH_E_INVALID, "obstacle radius");
    double an = std::sqrt(ob->axis[0] * ob->axis[0] + ob->axis[1] * ob->axis[1] + ob->axis[2] * ob->axis[2]);
    if (ob->kind == CLOTH_CYLINDER && !(an > 0)) return fail(CLOTH_E_INVALID, "cylinder axis");
    ObstD o{};
    o.kind = ob->kind;
    for (int i = 0; i < 3; ++i) {
        o.c[i] = ob->center[i];
        o.a[i] = an > 0 ? ob->axis[i] / an : (i == 0 ? 1.0 : 0.0);
    }
    o.R = ob->radius;
    o.wh = ob->omega * s.h;
    cloth_status rc = drop_graph(s);
    if (rc != CLOTH_OK) return rc;
    s.obst.push_back(o);
    return contact_set_obstacles(s, sc->c);
}

cloth_status cloth_set_state(cloth_scene sc, const float* x, const float* v, void* stream) {
    if (!sc || !x) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> t;
    aos_to_soa(x, t, s.nv, s.perm);
    HIPCHECK(hipMemcpyAsync(s.d.x, t.data(), sizeof(float) * 3 * s.nv, hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (v) {
        aos_to_soa(v, t, s.nv, s.perm);
        HIPCHECK(hipMemcpyAsync(s.d.v, t.data(), sizeof(float) * 3 * s.nv, hipMemcpyHostToDevice, st));
    } else {
        HIPCHECK(hipMemsetAsync(s.d.v, 0, sizeof(float) * 3 * s.nv, st));
    }
    // a new state starts without a forwarded residual and with a clear
    // overflow record
    HIPCHECK(hipMemsetAsync(s.d_rfdx, 0, sizeof(float) * 3 * s.nv, st));
    cloth_status rc = contact_reset(s, sc->c, st);
    if (rc != CLOTH_OK) return rc;
    HIPCHECK(hipStreamSynchronize(st));
    return CLOTH_OK;
}

cloth_status cloth_get_state(cloth_scene sc, float* x, float* v, void* stream) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> t(3 * (size_t)s.nv);
    if (x) {
        HIPCHECK(hipMemcpyAsync(t.data(), s.d.x, sizeof(float) * 3 * s.nv, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        soa_to_aos(t, x, s.nv, s.perm);
    }
    if (v) {
        HIPCHECK(hipMemcpyAsync(t.data(), s.d.v, sizeof(float) * 3 * s.nv, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        soa_to_aos(t, v, s.nv, s.perm);
    }
    return CLOTH_OK;
}

static cloth_status step_enqueue(cloth_scene sc, const float g[3], hipStream_t st) {
    Scene& s = sc->s;
    ContactState& c = sc->c;
    Dev& d = s.d;
    const int n = s.nv;
    // tolerance mode: the loop conditions of Algorithm 1 are decided on the
    // device before each inner iteration (k_gate); the launches of a skipped
    // iteration or block see a set gate and do nothing
    const bool tol = s.tol_in > 0 || s.tol_out > 0;
    // the gate is set only around the launches of one iteration or block end;
    // an early return must not leave it set for later launches
    struct GateReset {
        Dev& d;
        ~GateReset() { d.gate = nullptr; }
    } gate_reset{d};
    d.gate = nullptr;
    TIMED(K_MISC, launch_step_open(d.dxbits, s.nslots_cap, c.cnt, s.d_gate, st));
    const bool contact = contact_enabled(s, c);
    const bool rf = s.rf_iters > 0 && contact;
    TIMED(K_PREDICT, launch_predict(d, (float)s.h, g[0], g[1], g[2], rf ? s.d_rfdx : nullptr, st));
    const float* xplus = d.z;
    if (s.warm_iters > 0) {
        TIMED(K_MISC, launch_copy3(d.xk, d.z, n, st));
        for (int i = 0; i < s.warm_iters; ++i) {
            cloth_status rc = modal_iteration(sc, st);
            if (rc != CLOTH_OK) return rc;
        }
        xplus = d.xk;
    }
    if (contact) {
        // x- = x*, x+: CCD, filter -> x, x- (timed by phase inside)
        cloth_status rc = contact_step_begin(s, c, xplus, st);
        if (rc != CLOTH_OK) return rc;
    } else {
        TIMED(K_MISC, launch_copy3(d.x, xplus, n, st));
    }
    for (int o = 0; o < s.iters_out; ++o) {
        TIMED(K_MISC, launch_copy3(d.xk, d.x, n, st));
        TIMED(K_MISC, launch_copy3(d.xkm1, d.x, n, st));
        bool tready = false;   // the pair targets of iteration k are written
        for (int k = 0; k < s.iters_in; ++k) {
            const int slot = slot_inner(s, o, k);
            if (tol) {
                TIMED(K_MISC, launch_gate(s.d_gate, d.dxbits, k > 0 ? slot - 1 : -1, s.tol_in,
                                          o > 0 ? slot_outer(s, o - 1) : -1, s.tol_out, 1, c.cnt, st));
                d.gate = s.d_gate;
            }
            cloth_status rc = inner_iteration(sc, k, slot, st, false, 0.f, false, slot > 0 ? slot - 1 : -1, tready);
            // within a block the partial CCD also writes the next iteration's
            // pair targets (one launch less per iteration)
            const bool fuse = k + 1 < s.iters_in;
            if (rc == CLOTH_OK && contact) TIMED(K_PCCD, contact_partial_ccd(s, c, st, fuse));
            tready = contact && fuse && s.self_contact && c.active;
            d.gate = nullptr;
            if (rc != CLOTH_OK) return rc;
        }
        // the block's end (its gate: the outer condition of its first iteration)
        if (tol) d.gate = s.d_gate + 1;
        unsigned long long* dxo = dx_slot(s, slot_outer(s, o));
        if (contact) {
            bool last = o == s.iters_out - 1;
            cloth_status rc = contact_block_end(s, c, !last || rf, dxo, st);  // x+ = x^k -> x, x-
            if (rc != CLOTH_OK) return rc;
        } else {
            TIMED(K_MISC, launch_block_end(d, dxo, st));
        }
        d.gate = nullptr;
    }
    if (rf) {
        // residual forwarding (section 6): collision weights at k, no filter;
        // the displacement is kept only if the exiting t_TOI was small
        TIMED(K_MISC, launch_copy3(d.xk, d.x, n, st));
        TIMED(K_MISC, launch_copy3(d.xkm1, d.x, n, st));
        for (int k = 0; k < s.rf_iters; ++k) {
            const int slot = slot_rf(s, k);
            if (s.tol_in > 0) {
                TIMED(K_MISC, launch_gate(s.d_gate, d.dxbits, k > 0 ? slot - 1 : -1, s.tol_in, -1, 0.0, 0, c.cnt, st));
                d.gate = s.d_gate;
            }
            cloth_status rc = inner_iteration(sc, k, slot, st, false, 0.f, true, k > 0 ? slot - 1 : -1);
            d.gate = nullptr;
            if (rc != CLOTH_OK) return rc;
        }
        TIMED(K_MISC, launch_rf_finish(d, d.xk, d.x, s.d_rfdx, c.tmin_bits + 2, s.rf_toi, st));
    }
    if (s.debug_tangles) TIMED(K_MISC, contact_tangle_check(s, c, d.x, st));
    TIMED(K_MISC, launch_epilogue(d, (float)(1.0 / s.h), c.cnt, st));
    return CLOTH_OK;
}

// Records one step's launches into a graph (every count the kernels need is
// read from device memory, so the launch sequence of a step never changes).
}  // extern "C"

namespace cloth {
// Records one step's launches (with gravity g) into a new graph.
cloth_status record_step_graph(cloth_scene_s* sc, const float g[3], hipGraph_t* out) {
    Scene& s = sc->s;
    *out = nullptr;
    if (!s.cap_stream) HIPCHECK(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
    HIPCHECK(hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal));
    const bool timing = s.timing;
    s.timing = false;   // no timing events inside a graph
    cloth_status rc = step_enqueue(sc, g, s.cap_stream);
    s.timing = timing;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s.cap_stream, &graph);
    if (rc != CLOTH_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(CLOTH_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    *out = graph;
    return CLOTH_OK;
}
}  // namespace cloth

extern "C" {

static cloth_status capture_step(cloth_scene sc, const float g[3]) {
    Scene& s = sc->s;
    if (s.graph_exec) {
        HIPCHECK(hipGraphExecDestroy(s.graph_exec));
        s.graph_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    cloth_status rc = record_step_graph(sc, g, &graph);
    if (rc != CLOTH_OK) return rc;
    hipError_t e = hipGraphInstantiate(&s.graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(CLOTH_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    for (int i = 0; i < 3; ++i) s.graph_g[i] = g[i];
    return CLOTH_OK;
}

}  // extern "C"

namespace cloth {
// the scene's step graph, recorded for gravity g if needed
cloth_status prepare_step_graph(cloth_scene_s* sc, const float g[3]) {
    Scene& s = sc->s;
    if (!s.graph_exec || g[0] != s.graph_g[0] || g[1] != s.graph_g[1] || g[2] != s.graph_g[2])
        return capture_step(sc, g);
    return CLOTH_OK;
}
cloth_status scene_stats(cloth_scene_s* sc, hipStream_t st, cloth_step_stats* out);
}  // namespace cloth

extern "C" {

static cloth_status collect_stats(cloth_scene sc, hipStream_t st, cloth_step_stats* stats) {
    Scene& s = sc->s;
    ContactState& c = sc->c;
    const bool tol = s.tol_in > 0 || s.tol_out > 0;
    int h[CNT_TANGLES + 2];
    HIPCHECK(hipMemcpyAsync(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    std::vector<unsigned long long> bits = read_slots(s, s.nslots_cap, st);
    auto as_d = [](unsigned long long b) {
        double v;
        std::memcpy(&v, &b, 8);
        return v;
    };
    cloth_step_stats out{};
    out.inner_iters = tol ? h[CNT_INNER_DONE] : s.iters_in * s.iters_out;
    out.outer_iters = tol ? h[CNT_OUTER_DONE] : s.iters_out;
    // a skipped iteration repeats the norm of the last one that ran
    out.dx_norm = as_d(bits[slot_inner(s, s.iters_out - 1, s.iters_in - 1)]);
    out.outer_dx = as_d(bits[slot_outer(s, std::max(out.outer_iters, 1) - 1)]);
    out.cheb_rho = s.rho;
    out.cheb_gamma = s.gamma;
    out.min_toi = NO_HIT;
    cloth_status rc = contact_stats(s, c, st, &out);
    if (rc != CLOTH_OK) return rc;
    s.last = out;
    if (stats) *stats = out;
    const int fail_bits = h[CNT_STICKY];
    if (fail_bits) {
        // reported once: the record restarts empty
        HIPCHECK(hipMemsetAsync(c.cnt + CNT_STICKY, 0, sizeof(int), st));
        HIPCHECK(hipStreamSynchronize(st));
        std::string why = step_failure_text(s, c, fail_bits);
        if (fail_bits & STEP_TANGLED)
            why += " last check: " + std::to_string(h[CNT_TANGLES]) + " crossing edge-triangle pairs, " +
                   std::to_string(h[CNT_TANGLES + 1]) + " undecided;";
        const cloth_status code = (fail_bits & STEP_DIVERGED)  ? CLOTH_E_DIVERGED
                                  : (fail_bits & STEP_TANGLED) ? CLOTH_E_TANGLED
                                                               : CLOTH_E_CAPACITY;
        return fail(code, "a step since the last check failed and was rolled back:" + why);
    }
    return CLOTH_OK;
}

}  // extern "C"

namespace cloth {
cloth_status scene_stats(cloth_scene_s* sc, hipStream_t st, cloth_step_stats* out) {
    return collect_stats(sc, st, out);
}
}  // namespace cloth

extern "C" {

cloth_status cloth_step(cloth_scene sc, const float gravity[3], void* stream, cloth_step_stats* stats) {
    return cloth_step_n(sc, gravity, 1, stream, stats);
}

cloth_status cloth_step_n(cloth_scene sc, const float gravity[3], int32_t n, void* stream,
                          cloth_step_stats* stats) {
    if (!sc || !gravity) return fail(CLOTH_E_INVALID, "null argument");
    if (!sc->s.basis_set) return fail(CLOTH_E_INVALID, "basis not set");
    if (n < 0) return fail(CLOTH_E_INVALID, "negative step count");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scene& s = sc->s;
    bool graph = s.use_graph && !s.timing && n > 0;
    if (graph && (!s.graph_exec || gravity[0] != s.graph_g[0] || gravity[1] != s.graph_g[1] ||
                  gravity[2] != s.graph_g[2])) {
        cloth_status rc = capture_step(sc, gravity);
        if (rc != CLOTH_OK) return rc;
    }
    for (int i = 0; i < n; ++i) {
        if (graph) {
            HIPCHECK(hipGraphLaunch(s.graph_exec, st));
        } else {
            cloth_status rc = step_enqueue(sc, gravity, st);
            if (rc != CLOTH_OK) return rc;
        }
    }
    if (stats) return collect_stats(sc, st, stats);
    return CLOTH_OK;
}

cloth_status cloth_set_timing(cloth_scene sc, int32_t on) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    HIPCHECK(hipDeviceSynchronize());
    s.ev_used.clear();
    s.kt_ms.assign(K_COUNT, 0.0);
    s.kt_n.assign(K_COUNT, 0);
    s.timing = on != 0;
    return CLOTH_OK;
}

cloth_status cloth_kernel_times(cloth_scene sc, int32_t max, char* names, double* total_ms, int64_t* launches,
                                int32_t* count) {
    if (!sc || !count) return fail(CLOTH_E_INVALID, "null argument");
    Scene& s = sc->s;
    HIPCHECK(hipDeviceSynchronize());
    t_collect(s);
    *count = K_COUNT;
    for (int i = 0; i < K_COUNT && i < max; ++i) {
        if (names) {
            std::strncpy(names + 32 * i, kKernelNames[i], 31);
            names[32 * i + 31] = 0;
        }
        if (total_ms) total_ms[i] = s.kt_ms[i];
        if (launches) launches[i] = s.kt_n[i];
    }
    return CLOTH_OK;
}

cloth_status cloth_set_graph(cloth_scene sc, int32_t on) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    sc->s.use_graph = on != 0;
    return CLOTH_OK;
}

cloth_status cloth_destroy(cloth_scene sc) {
    if (!sc) return CLOTH_OK;
    if (sc->s.graph_exec) (void)hipGraphExecDestroy(sc->s.graph_exec);
    if (sc->s.cap_stream) (void)hipStreamDestroy(sc->s.cap_stream);
    for (hipEvent_t e : sc->s.ev_pool) (void)hipEventDestroy(e);
    if (sc->s.ev_fork) (void)hipEventDestroy(sc->s.ev_fork);
    if (sc->s.ev_join) (void)hipEventDestroy(sc->s.ev_join);
    if (sc->s.side) (void)hipStreamDestroy(sc->s.side);
    contact_destroy(sc->s, sc->c);
    if (sc->s.arena_owned) (void)hipFree(sc->s.arena);
    delete sc;
    return CLOTH_OK;
}

// Largest eigenvalue of D^{-1} H on the free rows (FP64 power iteration on
// the host copy of H): damped Jacobi x <- x + gamma D^{-1} r converges only
// for gamma < 2 / lambda_max.
static double jacobi_lambda_max(const Scene& s) {
    const int n = s.nv;
    std::vector<double> e(n), f(n);
    uint64_t st64 = 0x2545F4914F6CDD1Dull;
    for (int v = 0; v < n; ++v) {
        st64 ^= st64 << 13;
        st64 ^= st64 >> 7;
        st64 ^= st64 << 17;
        e[v] = s.pinned[v] ? 0.0 : (double)(st64 >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    double lam = 0.0;
    for (int it = 0; it < 150; ++it) {
        double nrm = 0.0;
#pragma omp parallel for reduction(+ : nrm) schedule(static)
        for (int v = 0; v < n; ++v) {
            double acc = 0.0;
            if (!s.pinned[v]) {
                for (int j = s.rowptr[v]; j < s.rowptr[v + 1]; ++j) acc += s.val[j] * e[s.col[j]];
                acc /= s.diag[v];
            }
            f[v] = acc;
            nrm += acc * acc;
        }
        nrm = std::sqrt(nrm);
        if (!(nrm > 0)) break;
        lam = nrm;
        for (int v = 0; v < n; ++v) e[v] = f[v] / nrm;
    }
    return lam;
}

// Chebyshev parameters from the device iteration itself.  The damping
// candidates are fractions of the Jacobi stability limit 2 / lambda_max; for
// each, the growth rate of the error of the coarse-corrected damped Jacobi
// sweep (b = 0, no contact, omega = 1) is measured by power iteration on the
// device; the fastest converging gamma is kept and rho is set slightly above
// the measured rate (underestimating rho makes the Chebyshev iteration
// diverge, overestimating only slows it).
cloth_status cloth_estimate_chebyshev(cloth_scene sc, void* stream) {
    Scene& s = sc->s;
    Dev& d = s.d;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = s.nv;
    const int warm = 100, meas = 100;
    double lmax = jacobi_lambda_max(s);
    double gmax = lmax > 0 ? 2.0 / lmax : 1.0;
    std::vector<double> cands;
    if (s.gamma > 0) {
        cands.push_back(s.gamma);
    } else {
        for (double f : {0.95, 0.85, 0.75, 0.65, 0.55}) cands.push_back(std::min(1.0, f * gmax));
    }
    std::vector<float> e(3 * (size_t)n);
    uint64_t st64 = 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < e.size(); ++i) {
        st64 ^= st64 << 13;
        st64 ^= st64 >> 7;
        st64 ^= st64 << 17;
        int v = (int)(i % n);
        e[i] = s.pinned[v] ? 0.f : (float)((double)(st64 >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
    double best_rate = 1e300, best_gamma = cands[0];
    for (double gm : cands) {
        s.gamma = gm;
        HIPCHECK(hipMemcpyAsync(d.xk, e.data(), sizeof(float) * e.size(), hipMemcpyHostToDevice, st));
        HIPCHECK(launch_copy3(d.xkm1, d.xk, n, st));
        HIPCHECK(launch_fill_u64(d.dxbits, 0ull, (warm + meas + 1) * DX_STRIDE, st));
        for (int k = 0; k < warm + meas; ++k) {
            cloth_status rc = inner_iteration(sc, k, k, st, true, 1.0f);
            if (rc != CLOTH_OK) return rc;
        }
        std::vector<unsigned long long> bits = read_slots(s, warm + meas, st);
        double a, b;
        std::memcpy(&a, &bits[warm - 1], 8);
        std::memcpy(&b, &bits[warm + meas - 1], 8);
        double rate = (a > 0 && b >= 0) ? std::pow(b / a, 1.0 / meas) : 1e300;
        if (!std::isfinite(rate)) rate = 1e300;
        if (rate < best_rate) {
            best_rate = rate;
            best_gamma = gm;
        }
    }
    s.gamma = best_gamma;
    if (!(best_rate < 0.9999))
        return fail(CLOTH_E_DIVERGED, "no damping gives a converging Jacobi sweep (rate " +
                                          std::to_string(best_rate) + ", lambda_max " + std::to_string(lmax) + ")");
    if (s.rho <= 0) s.rho = std::min(0.9999, 1.0 - 0.8 * (1.0 - best_rate));
    return CLOTH_OK;
}

// ---------------------------------------------------------------- stages

cloth_status cloth_stage_load_block(cloth_scene sc, const float* xm, const float* xk, const float* xkm1,
                                    const float* z, int64_t n_vt, const int32_t* vt, const int32_t* a_vt,
                                    int64_t n_ee, const int32_t* ee, const int32_t* a_ee,
                                    const int32_t* ob_a) {
    if (!sc || !xm || !xk || !xkm1 || !z) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    Scene& s = sc->s;
    Dev& d = s.d;
    std::vector<float> t;
    aos_to_soa(xm, t, s.nv);
    HIPCHECK(hipMemcpy(d.xm, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d.x, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    // the block's start stands for the step's start (the friction slip)
    HIPCHECK(hipMemcpy(d.xstar, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    aos_to_soa(xk, t, s.nv);
    HIPCHECK(hipMemcpy(d.xk, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    s.x4_valid = false;
    aos_to_soa(xkm1, t, s.nv);
    HIPCHECK(hipMemcpy(d.xkm1, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    aos_to_soa(z, t, s.nv);
    HIPCHECK(hipMemcpy(d.z, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    cloth_status rc = contact_load_constraints(s, sc->c, n_vt, vt, a_vt, n_ee, ee, a_ee, ob_a);
    if (rc != CLOTH_OK) return rc;
    HIPCHECK(hipDeviceSynchronize());
    return CLOTH_OK;
}

cloth_status cloth_stage_inner(cloth_scene sc, int32_t k) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    if (!sc->s.basis_set) return fail(CLOTH_E_INVALID, "basis not set");
    HIPCHECK(launch_fill_u64(sc->s.d.dxbits, 0ull, DX_STRIDE, nullptr));
    cloth_status rc = inner_iteration(sc, k, 0, nullptr, false, 0.f);
    if (rc != CLOTH_OK) return rc;
    if (sc->c.active) {
        rc = contact_partial_ccd(sc->s, sc->c, nullptr);
        if (rc != CLOTH_OK) return rc;
    }
    HIPCHECK(hipDeviceSynchronize());
    return CLOTH_OK;
}

cloth_status cloth_stage_partial_ccd(cloth_scene sc, const float* xnew) {
    if (!sc || !xnew) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    Scene& s = sc->s;
    if (!sc->c.active) return CLOTH_OK;
    std::vector<float> t;
    aos_to_soa(xnew, t, s.nv);
    HIPCHECK(hipMemcpy(s.d.xk, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    cloth_status rc = contact_partial_ccd(s, sc->c, nullptr);
    if (rc != CLOTH_OK) return rc;
    HIPCHECK(hipDeviceSynchronize());
    return CLOTH_OK;
}

cloth_status cloth_stage_read_block(cloth_scene sc, float* xk, int32_t* a_vt, int32_t* a_ee, int32_t* ob_a,
                                    double* dx, float* b, double* Q) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    Scene& s = sc->s;
    Dev& d = s.d;
    std::vector<float> t(3 * (size_t)s.nv);
    if (xk) {
        HIPCHECK(hipMemcpy(t.data(), d.xk, 12 * (size_t)s.nv, hipMemcpyDeviceToHost));
        soa_to_aos(t, xk, s.nv);
    }
    if (b) {
        HIPCHECK(hipMemcpy(t.data(), d.b, 12 * (size_t)s.nv, hipMemcpyDeviceToHost));
        soa_to_aos(t, b, s.nv);
    }
    if (Q) HIPCHECK(hipMemcpy(Q, d.Qd, sizeof(double) * 3 * s.r, hipMemcpyDeviceToHost));
    if (dx) {
        HIPCHECK(hipDeviceSynchronize());
        std::vector<unsigned long long> bits = read_slots(s, 1, nullptr);
        std::memcpy(dx, &bits[0], 8);
    }
    return contact_read_constraints(s, sc->c, a_vt, a_ee, ob_a);
}

cloth_status cloth_stage_outer(cloth_scene sc, const float* xm, const float* xp, int32_t first, float* x_out,
                               double* s_out) {
    if (!sc || !xm || !xp) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    return contact_stage_outer(sc->s, sc->c, xm, xp, first, x_out, s_out);
}

cloth_status cloth_stage_read_set(cloth_scene sc, int64_t cap, int32_t* vt, int32_t* a_vt, int64_t* n_vt,
                                  int32_t* ee, int32_t* a_ee, int64_t* n_ee, int32_t* ob_a) {
    if (!sc) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    return contact_stage_read_set(sc->s, sc->c, cap, vt, a_vt, n_vt, ee, a_ee, n_ee, ob_a);
}

cloth_status cloth_stage_broad_phase(cloth_scene sc, const float* xm, const float* xp, int64_t cap, int32_t* vt,
                                     int64_t* n_vt, int32_t* ee, int64_t* n_ee) {
    if (!sc || !xm || !xp || !n_vt || !n_ee) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    return contact_stage_broad_phase(sc->s, sc->c, xm, xp, cap, vt, n_vt, ee, n_ee);
}

cloth_status cloth_stage_toi(cloth_scene sc, const float* xm, const float* xp, int64_t n_vt, const int32_t* vt,
                             int64_t n_ee, const int32_t* ee, double* toi_vt, double* toi_ee) {
    if (!sc || !xm || !xp) return fail(CLOTH_E_INVALID, "null argument");
    if (reordered(sc->s)) return fail(CLOTH_E_INVALID, "stage calls need a scene in the caller's vertex order");
    return contact_stage_toi(sc->s, sc->c, xm, xp, n_vt, vt, n_ee, ee, toi_vt, toi_ee);
}

}  // extern "C"

namespace cloth {
cloth_status set_error(cloth_status code, const std::string& msg) { return fail(code, msg); }
}  // namespace cloth
