// Autotuner of the step's launch settings whose results are bitwise the same
// whatever they are, so that a setting is chosen on time alone at equal
// accuracy:
//   * lanes per broad-phase query (4, 8 or 16): how the counting and writing
//     passes spread a query over a wavefront;
//   * for scenes created with broad_reuse: the reusable candidate superset
//     on or off and its growth margins.
// The Chebyshev schedule (rho, damping) is picked on the device when the
// basis is set, by measured error growth (cloth_estimate_chebyshev); the
// tuner reports it.  Trials step the scene from its current state with each
// candidate setting (one untimed step, then `steps` timed steps between HIP
// events on the caller's stream), restoring the state between trials, and
// the fastest setting is kept and cached per size class (vertex count to a
// quarter octave, basis width, precision, self contact), so that later
// scenes of the same class take it without trials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "contact.hpp"
#include "scene.hpp"

namespace cloth {
cloth_status scene_drop_graph(cloth_scene_s* sc);   // api.cpp
}  // namespace cloth

using namespace cloth;

namespace {

using Key = std::tuple<int, int, int, int>;

std::mutex g_mu;
std::map<Key, cloth_tuning> g_cache;

Key class_of(const Scene& s) {
    const int bucket = (int)std::lround(4.0 * std::log2((double)std::max(1, s.nv)));
    return Key(bucket, s.r, s.prec, s.self_contact);
}

cloth_status apply(cloth_scene_s* sc, const cloth_tuning& t) {
    ContactState& c = sc->c;
    if (t.query_lanes != 4 && t.query_lanes != 8 && t.query_lanes != 16)
        return set_error(CLOTH_E_INVALID, "query_lanes must be 4, 8 or 16");
    if (t.broad_reuse && !sc->s.bp_reuse)
        return set_error(CLOTH_E_INVALID, "broad_reuse needs a scene created with broad_reuse");
    c.qlanes = t.query_lanes;
    c.sup_on = t.broad_reuse != 0 && sc->s.bp_reuse;
    if (t.broad_margin > 0) c.sup_mu0 = t.broad_margin;
    if (t.broad_margin_motion > 0) c.sup_kappa = t.broad_margin_motion;
    return scene_drop_graph(sc);
}

}  // namespace

extern "C" {

cloth_status cloth_set_tuning(cloth_scene sc, const cloth_tuning* t) {
    if (!sc || !t) return set_error(CLOTH_E_INVALID, "null argument");
    return apply(sc, *t);
}

cloth_status cloth_autotune(cloth_scene sc, const float gravity[3], int32_t steps, int32_t force, void* stream,
                            cloth_tuning* out) {
    if (!sc || !gravity || steps <= 0) return set_error(CLOTH_E_INVALID, "invalid argument");
    if (!sc->s.basis_set) return set_error(CLOTH_E_INVALID, "basis not set");
    Scene& s = sc->s;
    ContactState& c = sc->c;
    const Key key = class_of(s);
    if (!force) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            cloth_tuning t = it->second;
            t.from_cache = 1;
            t.trials = 0;
            t.cheb_rho = s.rho;
            t.cheb_gamma = s.gamma;
            cloth_status rc = apply(sc, t);
            if (rc != CLOTH_OK) return rc;
            if (out) *out = t;
            return CLOTH_OK;
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the candidates: lanes per query, then (scenes with a superset) the
    // superset with the default and a wider margin
    std::vector<cloth_tuning> cand;
    auto base = [&]() {
        cloth_tuning t{};
        t.query_lanes = 8;
        t.broad_reuse = 0;
        t.broad_margin = s.bp_mu0;
        t.broad_margin_motion = s.bp_kappa;
        return t;
    };
    for (int g : {8, 4, 16}) {
        cloth_tuning t = base();
        t.query_lanes = g;
        cand.push_back(t);
    }
    if (s.bp_reuse && s.self_contact)
        for (double m : {1.0, 2.0}) {
            cloth_tuning t = base();
            t.broad_reuse = 1;
            t.broad_margin = m * s.bp_mu0;
            cand.push_back(t);
        }
    // the state to return to between trials
    std::vector<float> x((size_t)3 * s.nv), v((size_t)3 * s.nv);
    cloth_status rc = cloth_get_state(sc, x.data(), v.data(), stream);
    if (rc != CLOTH_OK) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(CLOTH_E_DEVICE, "hipEventCreate");
    const cloth_tuning keep{c.qlanes, c.sup_on ? 1 : 0, c.sup_mu0, c.sup_kappa};
    double best_ms = 1e300, default_ms = 0.0;
    int best = 0;
    for (size_t i = 0; i < cand.size() && rc == CLOTH_OK; ++i) {
        rc = apply(sc, cand[i]);
        if (rc == CLOTH_OK) rc = cloth_set_state(sc, x.data(), v.data(), stream);
        if (rc == CLOTH_OK) rc = cloth_step_n(sc, gravity, 1, stream, nullptr);   // records the graph
        if (rc != CLOTH_OK) break;
        (void)hipEventRecord(e0, st);
        rc = cloth_step_n(sc, gravity, steps, stream, nullptr);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) rc = set_error(CLOTH_E_DEVICE, "hipEventSynchronize");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = ms / steps;
        if (i == 0) default_ms = per;
        if (per < best_ms) {
            best_ms = per;
            best = (int)i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // a failed step of a trial (a capacity, say) is reported by the next
    // stats read; the state goes back either way
    cloth_status rs = cloth_set_state(sc, x.data(), v.data(), stream);
    if (rc != CLOTH_OK) {
        (void)apply(sc, keep);
        return rc;
    }
    if (rs != CLOTH_OK) return rs;
    cloth_tuning t = cand[best];
    t.ms_per_step = best_ms;
    t.ms_default = default_ms;
    t.trials = (int)cand.size();
    t.from_cache = 0;
    t.cheb_rho = s.rho;
    t.cheb_gamma = s.gamma;
    rc = apply(sc, t);
    if (rc != CLOTH_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = t;
    }
    if (out) *out = t;
    return CLOTH_OK;
}

}  // extern "C"
