// Contact side of the cloth step: broad phase, time of impact, constraint
// sets with life spans, NDB weights and targets, partial CCD, the reduced
// matrix update U^T diag(W) U and its FP64 factorisation on the device.
#pragma once

#include <functional>

#include "scene.hpp"

namespace cloth {

// Broad-phase grids of one target family (cell widths of the fine grid 1
// and the coarse grid 2) and the inline record of a target in its bucket.
struct BpGrid {
    double cs1[3], cs2[3];   // cell width per axis
    int ok;                  // all extents finite
    int use2;                // some target is wider than a grid-1 cell
};

struct BpRec {
    long long key;             // grid (bit 63) and packed low-corner cell (21 bits per axis)
    int id, a, b, c;           // target id, its vertices (c = -1 for edges)
    float lo[3], hi[3];
};
static_assert(sizeof(BpRec) == 48, "BpRec layout");

struct ContactState {
    bool enabled = false;   // self contact or obstacles present
    bool active = false;    // the current block has constraints (or may have)
    int nob = 0;
    ObstD ob[MAX_OBST];
    int64_t cap = 0;        // candidate capacity per list (VT, EE)
    int64_t ccap = 0;       // constraint capacity (VT + EE together)
    int hash_p = 0;         // hash buckets (power of two)
    int max_out = 1024;     // candidate pairs one query may produce
    int ntiles_cap = 0;     // scan tiles for the largest scan

    // boxes (lo xyz, hi xyz as 6 floats)
    float *vbox = nullptr, *tbox = nullptr, *ebox = nullptr;
    int *bucket_cnt = nullptr, *bucket_ptr = nullptr;
    BpRec* rec = nullptr;   // targets in cell-bucket order
    int* qscratch = nullptr;  // per query: up to QK target ids from the counting pass
    int* heavy_q = nullptr;   // the queries with more than QK hits (counting pass -> rescan)
    float* bpart = nullptr;   // per-block box extents
    BpGrid* grid = nullptr;   // [0] triangles, [1] edges
    float4 *xm4 = nullptr, *xp4 = nullptr;   // AoS copies of the stage's two positions (TOI gathers)
    // reusable candidate superset: grown boxes, its sorted pairs, its words
    // (see k_sup_gate) and the growth margins
    float *svbox = nullptr, *stbox = nullptr, *sebox = nullptr;
    int2 *sup_vt = nullptr, *sup_ee = nullptr;
    int* toi_sched = nullptr;   // TOI chunk counters, one per XCD range on its own line
    int* supw = nullptr;
    double sup_mu0 = 0.0, sup_kappa = 1.0;
    bool sup_on = false;   // candidate lists filtered from the superset (else queried per stage)
    int qlanes = 8;        // lanes per broad-phase query (4, 8 or 16; the autotuner's choice)

    // candidates
    int* vcount = nullptr;  // per vertex VT counts, then offsets (nv+1)
    int* ecount = nullptr;  // per edge EE counts, then offsets (ne+1)
    int2 *cand_vt = nullptr, *cand_ee = nullptr;
    double *toi_vt = nullptr, *toi_ee = nullptr;
    int *keep = nullptr, *keep_ofs = nullptr, *cand_a = nullptr;

    // constraints (VT first, then EE), current and previous block
    int2 *cpair = nullptr, *cpair_prev = nullptr;
    int *ca = nullptr, *ca_prev = nullptr;
    double2* clam = nullptr;
    float4* cnrm = nullptr;
    float4* slot = nullptr;      // 4 per constraint: (w, w*y)
    int *vslot_ptr = nullptr, *vslot = nullptr, *vslot_fill = nullptr;
    int* ob_a = nullptr;         // MAX_OBST * nv, -1 = not a member
    int* cvlist = nullptr;       // contact vertices (for the Gram)
    int *cvflag = nullptr, *cvofs = nullptr;
    ObstD* ob_dev = nullptr;     // device copy of ob[]

    // device scalars: [0] n_vt cand, [1] n_ee cand, [2] n_cvt, [3] n_cee,
    // [4] n_prev_vt, [5] n_prev_ee, [6] n_cv, [7] status bits of the running
    // step (capacity overflows, divergence), [12] largest candidate list
    // since the last stats read, [9] n_vt + n_ee, [10] obstacle constraints,
    // [13] status bits since the last stats read, [14] the last step's
    // status, [15] / [16] inner iterations / outer blocks the step ran
    int* cnt = nullptr;
    unsigned long long* tmin_bits = nullptr;  // [0] stage min, [1] step min, [2] last stage's t_TOI
    double* tpart = nullptr;                  // per-block TOI minima of a stage (TOI, then obstacle blocks)
    double* s_dev = nullptr;                  // filter step length
    int64_t* stat64 = nullptr;                // [0] candidates (last), [1] constraints (last)

    // scan scratch
    int* scan_tiles = nullptr;
    double* gpart2 = nullptr;    // level-1 partials of U^T r0 (also used without contact)
    double* gvec = nullptr;      // g = U^T r0 (r*3, FP64)
    int gram_chunks = 0;
};

using Carver = std::function<void*(size_t)>;

// fills the per-vertex store of upper triangles of U_j U_j^T (Eq. (uu)) from
// the stored basis (synchronous)
cloth_status contact_build_uu(Scene& s);
// carves the contact buffers (a counting carver gives the footprint)
cloth_status contact_layout(Scene& s, ContactState& c, const Carver& carve);
cloth_status contact_upload(Scene& s, ContactState& c);
cloth_status contact_set_obstacles(Scene& s, ContactState& c);
bool contact_enabled(const Scene& s, const ContactState& c);
cloth_status contact_step_begin(Scene& s, ContactState& c, const float* xp, hipStream_t st);
cloth_status contact_block_begin(Scene& s, ContactState& c, hipStream_t st);
cloth_status contact_prepare_iteration(Scene& s, ContactState& c, bool force_k, hipStream_t st);
// the contact matrix and its factorization (needs only the weights: may
// run beside the local step), then q = A^{-1} g on it
cloth_status contact_factor(Scene& s, ContactState& c, bool force_k, hipStream_t st);
cloth_status contact_solve(Scene& s, ContactState& c, hipStream_t st);
// targets: also the pair constraints' targets of the next iteration (from
// the new life spans and x^k), so that it needs no k_pair_targets launch
cloth_status contact_partial_ccd(Scene& s, ContactState& c, hipStream_t st, bool targets = false);
// dxo: slot of the change of x over the block (the outer loop condition)
cloth_status contact_block_end(Scene& s, ContactState& c, bool setup, unsigned long long* dxo, hipStream_t st);
cloth_status contact_stats(Scene& s, ContactState& c, hipStream_t st, cloth_step_stats* out);
// debug tangle check of the positions x (sets STEP_TANGLED in the running
// step's status when an edge crosses a triangle sharing none of its vertices)
cloth_status contact_tangle_check(Scene& s, ContactState& c, const float* x, hipStream_t st);
// the reasons behind a failed step's status bits
std::string step_failure_text(const Scene& s, const ContactState& c, int bits);
// clears the sticky overflow record (with a new state)
cloth_status contact_reset(Scene& s, ContactState& c, hipStream_t st);
cloth_status contact_load_constraints(Scene& s, ContactState& c, int64_t n_vt, const int32_t* vt,
                                      const int32_t* a_vt, int64_t n_ee, const int32_t* ee,
                                      const int32_t* a_ee, const int32_t* ob_a);
cloth_status contact_read_constraints(Scene& s, ContactState& c, int32_t* a_vt, int32_t* a_ee,
                                      int32_t* ob_a);
cloth_status contact_stage_broad_phase(Scene& s, ContactState& c, const float* xm, const float* xp,
                                       int64_t cap, int32_t* vt, int64_t* n_vt, int32_t* ee,
                                       int64_t* n_ee);
cloth_status contact_stage_toi(Scene& s, ContactState& c, const float* xm, const float* xp,
                               int64_t n_vt, const int32_t* vt, int64_t n_ee, const int32_t* ee,
                               double* toi_vt, double* toi_ee);
cloth_status contact_stage_outer(Scene& s, ContactState& c, const float* xm, const float* xp, int first,
                                 float* x_out, double* s_out);
cloth_status contact_stage_read_set(Scene& s, ContactState& c, int64_t cap, int32_t* vt, int32_t* a_vt,
                                    int64_t* n_vt, int32_t* ee, int32_t* a_ee, int64_t* n_ee, int32_t* ob_a);
void contact_destroy(Scene& s, ContactState& c);

cloth_status set_error(cloth_status code, const std::string& msg);

}  // namespace cloth

// the opaque scene handle of the ABI
struct cloth_scene_s {
    cloth::Scene s;
    cloth::ContactState c;
};
