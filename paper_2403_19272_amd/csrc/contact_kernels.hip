// Contact kernels for gfx950: swept-box spatial hash broad phase, FP64
// time of impact, constraint sets with life spans (non-distance barrier,
// Eq. (exp)), partial CCD (Eq. (query)), half-space and obstacle targets,
// U^T diag(W) U over the contact vertices (Eq. (uu)) and a one-workgroup FP64
// Cholesky of the reduced matrix (Eq. (subspace_collision)).
//
// Every kernel takes its item counts from device memory and loops over them
// with a fixed grid, so the whole step can be enqueued without reading
// anything back on the host.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "contact.hpp"
#include "friction.hpp"
#include "kernels.hpp"

namespace cloth {

namespace {
// Launch carrying the timing events of a single-kernel timing bracket, if
// one is open on this thread (see timing_begin).
template <typename... KArgs, typename... Args>
void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args) {
    hipEvent_t a, b;
    if (kernel_events(&a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, a, b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
}
}  // namespace


// tolerance mode: a set gate turns the launch into a no-op (see Dev::gate)
__device__ __forceinline__ bool gated(const int* g) { return g && *g; }

namespace {

constexpr int SCAN_TILE = 2048;   // items per scan block (256 threads x 8)
constexpr int GRID_LOOP = 2048;   // blocks of the grid-stride kernels
constexpr int VT_SAMPLES = 3, EE_SAMPLES = 3;

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator*(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 lerp(d3 a, d3 b, double t) { return a + (b - a) * t; }
__device__ __forceinline__ d3 ld3(const float* X, int n, int v) {
    return {(double)X[v], (double)X[n + v], (double)X[2 * n + v]};
}
__device__ __forceinline__ double amax(d3 a) { return fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z))); }

__device__ __forceinline__ double warp_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// ---------------------------------------------------------------- TOI
// Earliest t in [0,1] at which the moving points are coplanar (cubic in t)
// and in contact; degenerate cubics fall back to sampled distances.
constexpr double DEGEN_REL = 1e-14, PAR_REL = 1e-20, NOHIT = 2.0;
constexpr int FALLBACK_SAMPLES = 1024;

__device__ double horner(const double c[4], double t) { return ((c[3] * t + c[2]) * t + c[1]) * t + c[0]; }
__device__ int sgnd(double v) { return (v > 0) - (v < 0); }

// Roots of the cubic in [0, 1] in increasing order: the interval is split
// at the critical points inside it; on each piece an endpoint value of 0 is
// a root, and a sign change is refined by bisection.  Each root is handed to
// `accept` in turn; the first one it accepts is returned (NOHIT if none).
// may_have_root01 runs the same bracketing without the refinement: false
// means the cubic has no root there, so the pair cannot hit.
struct Brackets {
    double brk[4];
    int nb;
};

__device__ __forceinline__ Brackets brackets01(const double c[4]) {
    Brackets r;
    r.brk[0] = 0.0;
    double A = 3 * c[3], B = 2 * c[2], C = c[1];
    double cr0 = 2.0, cr1 = 2.0;
    int ncr = 0;
    if (A != 0.0) {
        double disc = B * B - 4 * A * C;
        if (disc >= 0) {
            double sq = sqrt(disc);
            double q = -0.5 * (B + (B >= 0 ? sq : -sq));
            double r1 = q / A, r2 = (q != 0.0) ? C / q : r1;
            if (r1 > r2) {
                double t = r1;
                r1 = r2;
                r2 = t;
            }
            cr0 = r1;
            ncr = 1;
            if (r2 != r1) {
                cr1 = r2;
                ncr = 2;
            }
        }
    } else if (B != 0.0) {
        cr0 = -C / B;
        ncr = 1;
    }
    // breakpoints 0 < (critical points inside (0, 1), in order) < 1, written
    // with fixed indices so that they stay in registers
    const bool in0 = ncr >= 1 && cr0 > 0.0 && cr0 < 1.0, in1 = ncr >= 2 && cr1 > 0.0 && cr1 < 1.0;
    const int k = (int)in0 + (int)in1;
    const double e1 = in0 ? cr0 : cr1;
    r.brk[1] = k >= 1 ? e1 : 1.0;
    r.brk[2] = k >= 2 ? cr1 : 1.0;
    r.brk[3] = 1.0;
    r.nb = k + 2;
    return r;
}

__device__ bool may_have_root01(const double c[4]) {
    const Brackets br = brackets01(c);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i + 1 >= br.nb) break;
        double flo = horner(c, br.brk[i]), fhi = horner(c, br.brk[i + 1]);
        if (flo == 0.0 || fhi == 0.0 || sgnd(flo) != sgnd(fhi)) return true;
    }
    return false;
}

template <typename Accept>
__device__ double first_root01(const double c[4], Accept accept) {
    const Brackets br = brackets01(c);
    bool have_last = false;
    double last = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i + 1 >= br.nb) break;
        double lo = br.brk[i], hi = br.brk[i + 1];
        double flo = horner(c, lo), fhi = horner(c, hi);
        double root;
        if (flo == 0.0) {
            if (have_last && last == lo) continue;
            root = lo;
        } else if (fhi == 0.0) {
            root = hi;
        } else if (sgnd(flo) == sgnd(fhi)) {
            continue;
        } else {
            int s0 = sgnd(flo);
            for (int it = 0; it < 64; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = horner(c, mid);
                if (fm == 0.0) {
                    lo = mid;
                    break;
                }
                if (sgnd(fm) == s0) lo = mid; else hi = mid;
            }
            root = lo;
        }
        have_last = true;
        last = root;
        int verdict = accept(root);   // 1: hit at root, -1: stop (fallback taken), 0: next root
        if (verdict != 0) return verdict > 0 ? root : -1.0;
    }
    return NOHIT;
}

__device__ bool in_tri(d3 p, d3 a, d3 b, d3 c) {
    d3 n = cross(b - a, c - a);
    if (!(dot(n, n) > 0.0)) return false;
    return dot(cross(b - p, c - p), n) >= 0.0 && dot(cross(c - p, a - p), n) >= 0.0 &&
           dot(cross(a - p, b - p), n) >= 0.0;
}

// -1: parallel, 0: apart, 1: crossing (coplanar segments)
__device__ int seg_cross(d3 p1, d3 p2, d3 p3, d3 p4) {
    d3 d1 = p2 - p1, d2 = p4 - p3, r = p3 - p1;
    d3 n = cross(d1, d2);
    double nn = dot(n, n);
    if (nn <= PAR_REL * dot(d1, d1) * dot(d2, d2)) return -1;
    double s1 = dot(cross(r, d2), n) / nn, s2 = dot(cross(r, d1), n) / nn;
    return s1 >= 0.0 && s1 <= 1.0 && s2 >= 0.0 && s2 <= 1.0;
}

__device__ double clamp01(double v) { return v < 0 ? 0 : (v > 1 ? 1 : v); }

// closest point of triangle abc to p as (l1, l2): q = a + l1 (b-a) + l2 (c-a),
// by the Voronoi-region test of C. Ericson, Real-Time Collision Detection
// (2005), sec. 5.1.5 (the same operation order as the FP64 reference, so the
// frozen parameters agree bit for bit)
__device__ void tri_closest(d3 p, d3 a, d3 b, d3 c, double& l1, double& l2) {
    d3 ab = b - a, ac = c - a, ap = p - a;
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0 && d2 <= 0) { l1 = 0; l2 = 0; return; }
    d3 bp = p - b;
    double d3_ = dot(ab, bp), d4 = dot(ac, bp);
    if (d3_ >= 0 && d4 <= d3_) { l1 = 1; l2 = 0; return; }
    double vc = d1 * d4 - d3_ * d2;
    if (vc <= 0 && d1 >= 0 && d3_ <= 0) { l1 = d1 / (d1 - d3_); l2 = 0; return; }
    d3 cp = p - c;
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0 && d5 <= d6) { l1 = 0; l2 = 1; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) { l1 = 0; l2 = d2 / (d2 - d6); return; }
    double va = d3_ * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3_) >= 0 && (d5 - d6) >= 0) {
        double w = (d4 - d3_) / ((d4 - d3_) + (d5 - d6));
        l1 = 1 - w; l2 = w; return;
    }
    double den = va + vb + vc;
    if (den == 0.0) { l1 = 0; l2 = 0; return; }
    l1 = vb / den; l2 = vc / den;
}

// closest parameters (s on p1p2, t on p3p4): clamped line-line solution of
// C. Ericson, Real-Time Collision Detection (2005), sec. 5.1.9
__device__ void seg_closest(d3 p1, d3 p2, d3 p3, d3 p4, double& s, double& t) {
    d3 d1 = p2 - p1, d2 = p4 - p3, r = p1 - p3;
    double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    if (a <= 0 && e <= 0) { s = 0; t = 0; return; }
    if (a <= 0) { s = 0; t = clamp01(f / e); return; }
    double c = dot(d1, r);
    if (e <= 0) { t = 0; s = clamp01(-c / a); return; }
    double b = dot(d1, d2), den = a * e - b * b;
    s = den > 0 ? clamp01((b * f - c * e) / den) : 0.0;
    t = (b * s + f) / e;
    if (t < 0) { t = 0; s = clamp01(-c / a); }
    else if (t > 1) { t = 1; s = clamp01((b - c) / a); }
}

__device__ double dist_vt(const d3* q0, const d3* q1, double t) {
    d3 p = lerp(q0[0], q1[0], t), a = lerp(q0[1], q1[1], t), b = lerp(q0[2], q1[2], t), c = lerp(q0[3], q1[3], t);
    double l1, l2;
    tri_closest(p, a, b, c, l1, l2);
    d3 d = p - (a + (b - a) * l1 + (c - a) * l2);
    return sqrt(dot(d, d));
}
__device__ double dist_ee(const d3* q0, const d3* q1, double t) {
    d3 p1 = lerp(q0[0], q1[0], t), p2 = lerp(q0[1], q1[1], t), p3 = lerp(q0[2], q1[2], t), p4 = lerp(q0[3], q1[3], t);
    double s, u;
    seg_closest(p1, p2, p3, p4, s, u);
    d3 d = lerp(p3, p4, u) - lerp(p1, p2, s);
    return sqrt(dot(d, d));
}

template <bool VT>
__device__ double sampled_toi(const d3* q0, const d3* q1, double eta) {
    double prev = 0.0;
    for (int i = 0; i <= FALLBACK_SAMPLES; ++i) {
        double t = (double)i / FALLBACK_SAMPLES;
        double dd = VT ? dist_vt(q0, q1, t) : dist_ee(q0, q1, t);
        if (dd <= eta) {
            if (i == 0) return 0.0;
            double lo = prev, hi = t;
            for (int it = 0; it < 64; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double dm = VT ? dist_vt(q0, q1, mid) : dist_ee(q0, q1, mid);
                if (dm <= eta) hi = mid; else lo = mid;
            }
            return lo;
        }
        prev = t;
    }
    return NOHIT;
}

// The same fallback for one pair, taken by a whole wavefront: the samples
// are evaluated 64 at a time (lane l takes sample i0 + l) and the first one
// within eta is found with a ballot; the bisection that follows is the
// sequential one.  The result is bitwise that of sampled_toi: the same
// distances at the same parameters decide the same first sample.
template <bool VT>
__device__ double sampled_toi_wave(const d3* q0, const d3* q1, double eta, int lane) {
    int first = -1;
    for (int i0 = 0; i0 <= FALLBACK_SAMPLES && first < 0; i0 += 64) {
        const int i = i0 + lane;
        bool within = false;
        if (i <= FALLBACK_SAMPLES) {
            const double t = (double)i / FALLBACK_SAMPLES;
            within = (VT ? dist_vt(q0, q1, t) : dist_ee(q0, q1, t)) <= eta;
        }
        const unsigned long long m = __ballot(within);
        if (m) first = i0 + __ffsll((long long)m) - 1;
    }
    if (first < 0) return NOHIT;
    if (first == 0) return 0.0;
    double lo = (double)(first - 1) / FALLBACK_SAMPLES, hi = (double)first / FALLBACK_SAMPLES;
    for (int it = 0; it < 64; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double dm = VT ? dist_vt(q0, q1, mid) : dist_ee(q0, q1, mid);
        if (dm <= eta) hi = mid; else lo = mid;
    }
    return lo;
}

// coplanarity cubic of the points (p, a, b, c): ((b-a) x (c-a)) . (p-a)
__device__ void cubic_of(const d3* q0, const d3* q1, double c[4], double& L) {
    d3 E1 = q0[2] - q0[1], E2 = q0[3] - q0[1], W = q0[0] - q0[1];
    d3 F1 = q1[2] - q1[1], F2 = q1[3] - q1[1], Wf = q1[0] - q1[1];
    d3 dE1 = F1 - E1, dE2 = F2 - E2, dW = Wf - W;
    d3 C0 = cross(E1, E2), C1 = cross(E1, dE2) + cross(dE1, E2), C2 = cross(dE1, dE2);
    c[0] = dot(C0, W);
    c[1] = dot(C0, dW) + dot(C1, W);
    c[2] = dot(C1, dW) + dot(C2, W);
    c[3] = dot(C2, dW);
    L = fmax(fmax(fmax(amax(E1), amax(E2)), fmax(amax(W), amax(F1))), fmax(amax(F2), amax(Wf)));
}

__device__ bool degenerate(const double c[4], double L) {
    double s = fmax(fmax(fabs(c[0]), fabs(c[1])), fmax(fabs(c[2]), fabs(c[3])));
    return s <= DEGEN_REL * L * L * L;
}

// q: (vertex, a, b, c) at t=0 and t=1.  When the sampled fallback is
// needed, eta is set to its distance bound (> 0) and the return value is
// meaningless; otherwise eta is left at 0.
__device__ double pair_toi_vt(const d3* q0, const d3* q1, double& eta) {
    double c[4], L;
    cubic_of(q0, q1, c, L);
    if (L == 0.0) return NOHIT;
    if (degenerate(c, L)) {
        eta = 1e-12 * L;
        return NOHIT;
    }
    return first_root01(c, [&](double t) {
        return in_tri(lerp(q0[0], q1[0], t), lerp(q0[1], q1[1], t), lerp(q0[2], q1[2], t), lerp(q0[3], q1[3], t))
                   ? 1
                   : 0;
    });
}

__device__ __forceinline__ void ee_as_vt(const d3* e, d3* q) {
    q[0] = e[2];
    q[1] = e[0];
    q[2] = e[1];
    q[3] = e[0] + (e[3] - e[2]);
}

// e: (p1, p2, p3, p4) at t=0 and t=1; eta as for pair_toi_vt
__device__ double pair_toi_ee(const d3* e0, const d3* e1, double& eta) {
    d3 q0[4], q1[4];
    ee_as_vt(e0, q0);
    ee_as_vt(e1, q1);
    double c[4], L;
    cubic_of(q0, q1, c, L);
    if (L == 0.0) return NOHIT;
    if (degenerate(c, L)) {
        eta = 1e-12 * L;
        return NOHIT;
    }
    double t = first_root01(c, [&](double t) {
        int r = seg_cross(lerp(e0[0], e1[0], t), lerp(e0[1], e1[1], t), lerp(e0[2], e1[2], t), lerp(e0[3], e1[3], t));
        return r < 0 ? -1 : (r ? 1 : 0);
    });
    if (t < 0.0) eta = 1e-12 * L;
    return t;
}

// true when the pair certainly does not hit (the cubic has no root in
// [0, 1] and is not degenerate): the result is NOHIT without refinement
__device__ bool pair_no_hit(bool vt, const d3* p0, const d3* p1) {
    d3 q0[4], q1[4];
    if (vt) {
        for (int k = 0; k < 4; ++k) {
            q0[k] = p0[k];
            q1[k] = p1[k];
        }
    } else {
        ee_as_vt(p0, q0);
        ee_as_vt(p1, q1);
    }
    double c[4], L;
    cubic_of(q0, q1, c, L);
    if (L == 0.0) return true;
    if (degenerate(c, L)) return false;
    return !may_have_root01(c);
}

__device__ __forceinline__ void pair_points(const Dev& d, bool vt, int i, int j, const float* X, d3* q) {
    const int n = d.nv;
    if (vt) {
        TriRec tr = d.tri[j];
        q[0] = ld3(X, n, i);
        q[1] = ld3(X, n, tr.v0);
        q[2] = ld3(X, n, tr.v1);
        q[3] = ld3(X, n, tr.v2);
    } else {
        q[0] = ld3(X, n, d.edges[2 * i]);
        q[1] = ld3(X, n, d.edges[2 * i + 1]);
        q[2] = ld3(X, n, d.edges[2 * j]);
        q[3] = ld3(X, n, d.edges[2 * j + 1]);
    }
}

__device__ __forceinline__ d3 ld4(const float4* X4, int v) {
    float4 p = X4[v];
    return {(double)p.x, (double)p.y, (double)p.z};
}

// the pair's four points at both ends of the interval, from AoS copies
__device__ __forceinline__ void pair_points2(const Dev& d, bool vt, int i, int j, const float4* X0, const float4* X1,
                                             d3* q0, d3* q1) {
    int id[4];
    if (vt) {
        TriRec tr = d.tri[j];
        id[0] = i; id[1] = tr.v0; id[2] = tr.v1; id[3] = tr.v2;
    } else {
        int2 e = reinterpret_cast<const int2*>(d.edges)[i], f = reinterpret_cast<const int2*>(d.edges)[j];
        id[0] = e.x; id[1] = e.y; id[2] = f.x; id[3] = f.y;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        q0[k] = ld4(X0, id[k]);
        q1[k] = ld4(X1, id[k]);
    }
}

__device__ __forceinline__ void pair_ids(const Dev& d, bool vt, int i, int j, int* id) {
    if (vt) {
        TriRec tr = d.tri[j];
        id[0] = i; id[1] = tr.v0; id[2] = tr.v1; id[3] = tr.v2;
    } else {
        id[0] = d.edges[2 * i]; id[1] = d.edges[2 * i + 1]; id[2] = d.edges[2 * j]; id[3] = d.edges[2 * j + 1];
    }
}

// obstacle: signed distance and radial vector (FP64)
__device__ __forceinline__ double obst_phi(const ObstD& o, d3 x, d3& rv, double& rad) {
    d3 c = mk(o.c[0], o.c[1], o.c[2]);
    rv = x - c;
    if (o.kind == CLOTH_CYLINDER) {
        d3 a = mk(o.a[0], o.a[1], o.a[2]);
        rv = rv - a * dot(rv, a);
    }
    rad = sqrt(dot(rv, rv));
    return rad - o.R;
}

__device__ double obst_toi(const ObstD& o, d3 xm, d3 xp) {
    d3 dd = xp - xm, oo = xm - mk(o.c[0], o.c[1], o.c[2]);
    if (o.kind == CLOTH_CYLINDER) {
        d3 a = mk(o.a[0], o.a[1], o.a[2]);
        dd = dd - a * dot(dd, a);
        oo = oo - a * dot(oo, a);
    }
    double A = dot(dd, dd), B = 2 * dot(oo, dd), C = dot(oo, oo) - o.R * o.R;
    double disc = B * B - 4 * A * C;
    if (!(C > 0 && B < 0 && disc >= 0 && A > 0)) return NOHIT;
    double q = 0.5 * (-B + sqrt(disc));
    double t = C / q;
    return t <= 1.0 ? t : NOHIT;
}

}  // namespace

// ================================================================ scans
// Exclusive prefix sums over n = min(n_dev ? *n_dev : n_host, cap) ints.
// Within a wavefront the sums are formed with lane shuffles; one barrier
// per block combines the wavefront totals.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// tiles holding the first n items
__device__ __forceinline__ int scan_used_tiles(int n_host, const int* n_dev, int ntiles) {
    const int n = n_dev ? min(*n_dev, n_host) : n_host;
    return min(ntiles, (max(n, 0) + SCAN_TILE - 1) / SCAN_TILE);
}

// per-tile sums, tiles taken grid-stride
__global__ void __launch_bounds__(256) k_scan_tiles(const int* __restrict__ gate, const int* __restrict__ in, int n_host,
                                                    const int* __restrict__ n_dev, int ntiles, int* tiles) {
    if (gated(gate)) return;
    __shared__ int red[4];
    const int n = n_dev ? min(*n_dev, n_host) : n_host;
    const int used = scan_used_tiles(n_host, n_dev, ntiles);
    for (int tile = blockIdx.x; tile < used; tile += gridDim.x) {
        const int base = tile * SCAN_TILE;
        int s = 0;
        for (int i = threadIdx.x; i < SCAN_TILE; i += 256) {
            const int g = base + i;
            if (g < n) s += in[g];
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) tiles[tile] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();   // red is reused by the next tile
    }
}

// single block: exclusive scan of the used tile sums in place; total -> *total
__global__ void __launch_bounds__(1024) k_scan_top(const int* __restrict__ gate, int* tiles, int n_host, const int* __restrict__ n_dev, int ntiles,
                                                   int* total) {
    if (gated(gate)) return;
    __shared__ int wsum[16];
    const int used = scan_used_tiles(n_host, n_dev, ntiles);
    const int per = (used + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(used, b0 + per);
    int s = 0;
    for (int i = b0; i < b1; ++i) s += tiles[i];
    const int incl = wave_incl_scan(s);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    int run = woff + incl - s;
    for (int i = b0; i < b1; ++i) {
        const int t = tiles[i];
        tiles[i] = run;
        run += t;
    }
    if (threadIdx.x == 1023 && total) *total = woff + incl;
}

// items of each used tile, tiles taken grid-stride
__global__ void __launch_bounds__(256) k_scan_apply(const int* __restrict__ gate, const int* __restrict__ in, int n_host,
                                                    const int* __restrict__ n_dev, int ntiles,
                                                    const int* __restrict__ tiles, int* __restrict__ out) {
    if (gated(gate)) return;
    __shared__ int wsum[4];
    const int n = n_dev ? min(*n_dev, n_host) : n_host;
    const int used = scan_used_tiles(n_host, n_dev, ntiles);
    for (int tile = blockIdx.x; tile < used; tile += gridDim.x) {
        const int base = tile * SCAN_TILE;
        // each thread owns 8 consecutive items
        int v[8];
        int s = 0;
        for (int k = 0; k < 8; ++k) {
            const int g = base + threadIdx.x * 8 + k;
            v[k] = g < n ? in[g] : 0;
            s += v[k];
        }
        const int incl = wave_incl_scan(s);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 63) wsum[w] = incl;
        __syncthreads();
        int run = tiles[tile] + incl - s;
        for (int k = 0; k < w; ++k) run += wsum[k];
        for (int k = 0; k < 8; ++k) {
            const int g = base + threadIdx.x * 8 + k;
            if (g < n) out[g] = run;
            run += v[k];
        }
        __syncthreads();   // wsum is reused by the next tile
    }
}

// out[i] = exclusive prefix of in[0..i) for i < n = min(n_dev ? *n_dev : n_cap,
// n_cap) (out may not alias in); the grids are sized for n_cap and the
// kernels skip the tiles past n.
constexpr int SCAN_GRID = 1024;
static hipError_t scan_exclusive(const int* in, int* out, int n_cap, const int* n_dev, int* tiles, int* total,
                                 const int* gate, hipStream_t st) {
    int nt = (n_cap + SCAN_TILE - 1) / SCAN_TILE;
    if (nt == 0) nt = 1;
    const int grid = std::min(nt, SCAN_GRID);
    hipLaunchKernelGGL(k_scan_tiles, dim3(grid), dim3(256), 0, st, gate, in, n_cap, n_dev, nt, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, gate, tiles, n_cap, n_dev, nt, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid), dim3(256), 0, st, gate, in, n_cap, n_dev, nt, (const int*)tiles, out);
    return hipGetLastError();
}

// ================================================================ broad phase
//
// Candidate pairs are the pairs whose FP32 swept boxes (grown by d^) overlap;
// the structure below only has to find each of them once.  Targets
// (triangles for VT, edges for EE) are filed in the grid cell of their low
// corner, and a query box looks at the cells from one below its low corner
// to its high corner on every axis: every overlapping target is seen exactly
// once provided each target is narrower than a cell.  Two grids keep the
// cells small when a few boxes are much wider than the rest (fast-moving
// parts): grid 1 has cells of 3 x the mean target width per axis and holds
// the targets narrower than that; grid 2 has cells as wide as the widest
// target and holds the others (it is used only when such targets exist).
// Cells are hashed into one bucket table; each bucket holds inline records
// (packed grid + cell key, ids, box), so a query reads contiguous records
// and skips the ones of other cells that share its bucket.

__global__ void k_fill_i32(const int* __restrict__ gate, int* p, int v, int n) {
    if (gated(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// per block and family (triangles, edges): widest box, lowest and highest
// corner, sum of widths, per axis
constexpr int BP_FAM = 12;
constexpr int BP_PART = 2 * BP_FAM;
constexpr int QK = 48;        // candidates per query kept from the counting pass
constexpr int CELL_LIM = 1 << 20;   // |cell index| bound of the packed keys
constexpr double CELL_MARGIN = 1.0 + 1.0 / 1024.0;
// overflow flag bits (sticky until the host reads them)
constexpr int OVF_QUERY = 1, OVF_CELL = 2, OVF_LIST = 4, OVF_CONS = 8;
constexpr int PEAK_SLOT = 12;   // cnt[12]: largest candidate list since the last stats read
constexpr int HEAVY_SLOT = 25;  // cnt[25]: queries listed for k_query_rescan, cnt[26]: its workgroups done

__device__ __forceinline__ int bp_op(int k) { return (k % BP_FAM) / 3; }   // 0 max, 1 min, 2 max, 3 sum
__device__ __forceinline__ float bp_combine(int op, float a, float b) {
    return op == 1 ? fminf(a, b) : (op == 3 ? a + b : fmaxf(a, b));
}
__device__ __forceinline__ float bp_identity(int op) {
    return op == 1 ? INFINITY : (op == 2 ? -INFINITY : 0.f);
}

__device__ __forceinline__ unsigned hash3(int grid, int x, int y, int z) {
    return ((unsigned)x * 73856093u) ^ ((unsigned)y * 19349663u) ^ ((unsigned)z * 83492791u) ^
           (grid ? 0x9E3779B9u : 0u);
}
// Bucket of a cell: the 4 x 4 x 4 block of cells around it is hashed and the
// cell's place in its block picks one of 64 consecutive buckets, so that the
// cells a query scans (a 2..3-cell cube) lie in a few contiguous runs of the
// record array and neighbouring queries share cache lines.
__device__ __forceinline__ unsigned cell_bucket(int grid, int x, int y, int z, int P) {
    const unsigned in_block = (unsigned)(x & 3) | ((unsigned)(y & 3) << 2) | ((unsigned)(z & 3) << 4);
    return ((hash3(grid, x >> 2, y >> 2, z >> 2) << 6) | in_block) & (unsigned)(P - 1);
}
__device__ __forceinline__ long long cell_key(int grid, int x, int y, int z) {
    return ((long long)grid << 63) | ((long long)(x & 0x1FFFFF) << 42) | ((long long)(y & 0x1FFFFF) << 21) |
           (long long)(z & 0x1FFFFF);
}

// cell index along one axis, in FP64 so that the one-cell margin of the
// query range cannot be eaten by rounding; false for non-finite or far-away
// coordinates
__device__ __forceinline__ bool cell_d(float x, double cs, int& c) {
    double q = (double)x / cs;
    if (!(fabs(q) < (double)(CELL_LIM - 64))) return false;
    c = (int)floor(q);
    return true;
}

// cell of a point on grid `grid` of g (the cell sizes are selected per
// component: a pointer into a local grid struct would put it in scratch)
__device__ __forceinline__ bool cell3g(const float* lo, const BpGrid& g, int grid, int* c) {
    return cell_d(lo[0], grid ? g.cs2[0] : g.cs1[0], c[0]) && cell_d(lo[1], grid ? g.cs2[1] : g.cs1[1], c[1]) &&
           cell_d(lo[2], grid ? g.cs2[2] : g.cs1[2], c[2]);
}

// grid of a target box: 0 if narrower than a grid-1 cell on every axis
__device__ __forceinline__ int target_grid(const float* box, const BpGrid& g) {
    for (int a = 0; a < 3; ++a)
        if ((double)(box[3 + a] - box[a]) * CELL_MARGIN > g.cs1[a]) return 1;
    return 0;
}

// cell of a target: false (and cell 0 of grid 0) if it cannot be filed
__device__ __forceinline__ bool target_cell(const float* box, const BpGrid& g, int& grid, int* c) {
    grid = target_grid(box, g);
    if (g.ok && cell3g(box, g, grid, c)) return true;
    grid = 0;
    c[0] = c[1] = c[2] = 0;
    return false;
}

// AoS float4 copies of the two SoA position arrays (one 16-byte gather per
// corner in the boxes and the TOI)
__global__ void k_aos_pair(const int* __restrict__ gate, int n, const float* __restrict__ xm, const float* __restrict__ xp, float4* xm4,
                           float4* xp4) {
    if (gated(gate)) return;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        xm4[v] = make_float4(xm[v], xm[n + v], xm[2 * n + v], 0.f);
        xp4[v] = make_float4(xp[v], xp[n + v], xp[2 * n + v], 0.f);
    }
}

// Swept boxes over (xm, xp) grown by dhat (FP32); per block the box
// statistics of the triangle and edge boxes (reduced by k_grid).
__global__ void __launch_bounds__(256) k_boxes(Dev d, const float4* __restrict__ xm4, const float4* __restrict__ xp4,
                                               float dhat, float* vbox, float* tbox, float* ebox, float* bpart,
                                               const float* __restrict__ svbox, const float* __restrict__ stbox,
                                               const float* __restrict__ sebox, int* escaped) {
    if (gated(d.gate)) return;
    __shared__ float red[4][BP_PART];
    const int total = d.nv + d.nt + d.ne;
    float acc[BP_PART];
    for (int k = 0; k < BP_PART; ++k) acc[k] = bp_identity(bp_op(k));
    bool esc = false;   // a box not inside its reusable-list box (escaped != null)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        int ids[3];
        int nvert;
        float* out;
        int kind;
        if (i < d.nv) {
            ids[0] = i;
            nvert = 1;
            out = vbox + 6 * (size_t)i;
            kind = 0;
        } else if (i < d.nv + d.nt) {
            int t = i - d.nv;
            TriRec tr = d.tri[t];
            ids[0] = tr.v0; ids[1] = tr.v1; ids[2] = tr.v2;
            nvert = 3;
            out = tbox + 6 * (size_t)t;
            kind = 1;
        } else {
            int e = i - d.nv - d.nt;
            ids[0] = d.edges[2 * e];
            ids[1] = d.edges[2 * e + 1];
            nvert = 2;
            out = ebox + 6 * (size_t)e;
            kind = 2;
        }
        const float* sb = !escaped ? nullptr
                          : kind == 0 ? svbox + 6 * (size_t)i
                          : kind == 1 ? stbox + 6 * (size_t)(i - d.nv)
                                      : sebox + 6 * (size_t)(i - d.nv - d.nt);
        // the corners' two positions, one 16-byte load each
        float pa[3][3], pb[3][3];
        for (int k = 0; k < nvert; ++k) {
            const float4 a = xm4[ids[k]], b = xp4[ids[k]];
            pa[k][0] = a.x; pa[k][1] = a.y; pa[k][2] = a.z;
            pb[k][0] = b.x; pb[k][1] = b.y; pb[k][2] = b.z;
        }
        for (int c = 0; c < 3; ++c) {
            float lo = pa[0][c], hi = lo;
            for (int k = 0; k < nvert; ++k) {
                float a = pa[k][c], b = pb[k][c];
                lo = fminf(lo, fminf(a, b));
                hi = fmaxf(hi, fmaxf(a, b));
            }
            float l = lo - dhat, h = hi + dhat;
            out[c] = l;
            out[3 + c] = h;
            if (sb) esc |= !(l >= sb[c] && h <= sb[3 + c]);
            if (kind) {
                const int f = (kind - 1) * BP_FAM;
                acc[f + c] = fmaxf(acc[f + c], h - l);
                acc[f + 3 + c] = fminf(acc[f + 3 + c], l);
                acc[f + 6 + c] = fmaxf(acc[f + 6 + c], h);
                acc[f + 9 + c] += h - l;
            }
        }
    }
    if (escaped && __ballot(esc) && (threadIdx.x & 63) == 0) *escaped = 1;
    for (int k = 0; k < BP_PART; ++k) {
        const int op = bp_op(k);
        float w = acc[k];
        for (int o = 32; o > 0; o >>= 1) w = bp_combine(op, w, __shfl_xor(w, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < BP_PART) {
        const int k = threadIdx.x, op = bp_op(k);
        float w = red[0][k];
        for (int q = 1; q < 4; ++q) w = bp_combine(op, w, red[q][k]);
        bpart[(size_t)blockIdx.x * BP_PART + k] = w;
    }
}

// ---------------------------------------------------------- reusable lists
// The candidate lists of a stage are taken from a superset built on boxes
// grown by a margin, kept for as long as every stage box stays inside its
// grown box: then every pair whose stage boxes overlap has overlapping grown
// boxes and is in the superset, and filtering the (sorted) superset by the
// stage boxes gives exactly the sorted candidate lists.  The superset is
// rebuilt when a box leaves its grown box (checked in k_boxes).
// A superset on grown boxes can outgrow a capacity (a violent stage) where
// the candidate lists themselves fit: the rebuild is then done again at
// once on the stage boxes themselves (no margin).
// Words of ContactState::supw: [0] / [1] VT / EE superset sizes, [2] rebuild
// needed, [3] rebuilds since the last stats read, [4] superset size (VT +
// EE), [5] gate of the rebuild launches (1 = skip), [6] the gate of the
// stage (1 = skip) for the filter, [7] 1 = build without margins, [8] the
// step's overflow bits before the rebuild, [9] gate of the retry.

// gate of the rebuild: skipped when the stage is or the superset stands
__global__ void k_sup_gate(const int* __restrict__ stage_gate, int* supw, const int* __restrict__ cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int skip_stage = gated(stage_gate) ? 1 : 0;
        supw[5] = (skip_stage || !supw[2]) ? 1 : 0;
        supw[6] = skip_stage;
        supw[7] = 0;
        supw[8] = cnt[7];
        supw[9] = 1;
    }
}

// after the first rebuild: if it overflowed, forget those overflow bits and
// open the retry without margins
__global__ void k_sup_retry(int* supw, int* cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int mask = OVF_QUERY | OVF_CELL | OVF_LIST;
        if (!supw[5] && (cnt[7] & mask & ~supw[8])) {
            cnt[7] = supw[8];
            supw[7] = 1;
            supw[9] = 0;
        }
    }
}

// grown boxes: the stage box widened along axis c by min(mu0 + kappa m_c,
// 16 mu0), m_c the largest change of coordinate c of the primitive's corners
// over the stage, so that a box grows along its motion (a falling sheet
// keeps its neighbours in the plane) and the cap bounds the superset of a
// violent stage; per block the statistics of the grown triangle and edge
// boxes (for k_grid)
__global__ void __launch_bounds__(256) k_sup_grow(Dev d, const float4* __restrict__ xm4, const float4* __restrict__ xp4,
                                                  const float* __restrict__ vbox, const float* __restrict__ tbox,
                                                  const float* __restrict__ ebox, float* svbox, float* stbox,
                                                  float* sebox, float* bpart, float mu0, float kappa,
                                                  const int* __restrict__ exact) {
    if (gated(d.gate)) return;
    if (*exact) mu0 = kappa = 0.f;
    __shared__ float red[4][BP_PART];
    const int total = d.nv + d.nt + d.ne;
    float acc[BP_PART];
    for (int k = 0; k < BP_PART; ++k) acc[k] = bp_identity(bp_op(k));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        int ids[3];
        int nvert, kind;
        const float* in;
        float* out;
        if (i < d.nv) {
            ids[0] = i;
            nvert = 1;
            kind = 0;
            in = vbox + 6 * (size_t)i;
            out = svbox + 6 * (size_t)i;
        } else if (i < d.nv + d.nt) {
            const int t = i - d.nv;
            const TriRec tr = d.tri[t];
            ids[0] = tr.v0; ids[1] = tr.v1; ids[2] = tr.v2;
            nvert = 3;
            kind = 1;
            in = tbox + 6 * (size_t)t;
            out = stbox + 6 * (size_t)t;
        } else {
            const int e = i - d.nv - d.nt;
            ids[0] = d.edges[2 * e];
            ids[1] = d.edges[2 * e + 1];
            nvert = 2;
            kind = 2;
            in = ebox + 6 * (size_t)e;
            out = sebox + 6 * (size_t)e;
        }
        float m[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < nvert; ++k) {
            const float4 a = xm4[ids[k]], b = xp4[ids[k]];
            m[0] = fmaxf(m[0], fabsf(b.x - a.x));
            m[1] = fmaxf(m[1], fabsf(b.y - a.y));
            m[2] = fmaxf(m[2], fabsf(b.z - a.z));
        }
        for (int c = 0; c < 3; ++c) {
            const float mu = fminf(mu0 + kappa * m[c], 16.f * mu0);
            const float l = in[c] - mu, h = in[3 + c] + mu;
            out[c] = l;
            out[3 + c] = h;
            if (kind) {
                const int f = (kind - 1) * BP_FAM;
                acc[f + c] = fmaxf(acc[f + c], h - l);
                acc[f + 3 + c] = fminf(acc[f + 3 + c], l);
                acc[f + 6 + c] = fmaxf(acc[f + 6 + c], h);
                acc[f + 9 + c] += h - l;
            }
        }
    }
    for (int k = 0; k < BP_PART; ++k) {
        const int op = bp_op(k);
        float w = acc[k];
        for (int o = 32; o > 0; o >>= 1) w = bp_combine(op, w, __shfl_xor(w, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < BP_PART) {
        const int k = threadIdx.x, op = bp_op(k);
        float w = red[0][k];
        for (int q = 1; q < 4; ++q) w = bp_combine(op, w, red[q][k]);
        bpart[(size_t)blockIdx.x * BP_PART + k] = w;
    }
}

// after a rebuild: the superset stands unless a list overflowed (then the
// next stage rebuilds again)
__global__ void k_sup_done(const int* __restrict__ gate, int* supw, const int* __restrict__ cnt) {
    if (gated(gate)) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        supw[2] = (cnt[7] & (OVF_QUERY | OVF_CELL | OVF_LIST)) ? 1 : 0;
        supw[3] += 1;
    }
}

__device__ __forceinline__ bool boxes_overlap(const float* a, const float* b) {
    return !(a[0] > b[3] || b[0] > a[3] || a[1] > b[4] || b[1] > a[4] || a[2] > b[5] || b[2] > a[5]);
}

// keep[i] = 1 for the superset pairs (VT, then EE) whose stage boxes overlap
// (ids outside the mesh, possible only in a list cut short by an overflow,
// are dropped)
__global__ void __launch_bounds__(256) k_sup_filter(int* supw, const int2* __restrict__ svt,
                                                    const int2* __restrict__ see, const float* __restrict__ vbox,
                                                    const float* __restrict__ tbox, const float* __restrict__ ebox,
                                                    int nv, int nt, int ne, int* keep) {
    if (supw[6]) return;
    const int nvt = supw[0], tot = supw[0] + supw[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) supw[4] = tot;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
        bool k;
        if (i < nvt) {
            const int2 p = svt[i];
            k = (unsigned)p.x < (unsigned)nv && (unsigned)p.y < (unsigned)nt &&
                boxes_overlap(vbox + 6 * (size_t)p.x, tbox + 6 * (size_t)p.y);
        } else {
            const int2 p = see[i - nvt];
            k = (unsigned)p.x < (unsigned)ne && (unsigned)p.y < (unsigned)ne &&
                boxes_overlap(ebox + 6 * (size_t)p.x, ebox + 6 * (size_t)p.y);
        }
        keep[i] = k ? 1 : 0;
    }
}

// the kept pairs to the candidate lists (order kept), their counts in
// cnt[0], cnt[1] and the largest list in the peak slot; a list longer than
// the candidate capacity is cut there and flagged (the step then fails)
__global__ void __launch_bounds__(256) k_sup_compact(const int* __restrict__ supw, const int2* __restrict__ svt,
                                                     const int2* __restrict__ see, const int* __restrict__ keep,
                                                     const int* __restrict__ ofs, int2* cvt, int2* cee, int* cnt,
                                                     int64_t cap) {
    if (supw[6]) return;
    const int nvt = supw[0], tot = supw[0] + supw[1];
    const int kvt = nvt > 0 ? ofs[nvt - 1] + keep[nvt - 1] : 0;
    const int kall = tot > 0 ? ofs[tot - 1] + keep[tot - 1] : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int kee = kall - kvt;
        cnt[PEAK_SLOT] = max(cnt[PEAK_SLOT], max(kvt, kee));
        if (kvt > cap || kee > cap) atomicOr(&cnt[7], OVF_LIST);
        cnt[0] = (int)min((int64_t)kvt, cap);
        cnt[1] = (int)min((int64_t)kee, cap);
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
        if (!keep[i]) continue;
        if (i < nvt) {
            if (ofs[i] < cap) cvt[ofs[i]] = svt[i];
        } else if (ofs[i] - kvt < cap) {
            cee[ofs[i] - kvt] = see[i - nvt];
        }
    }
}

// per-query offsets of the candidate lists: the first entry of query q
// (lists sorted by query), for the vertices and then the edges
__global__ void __launch_bounds__(256) k_query_ofs(const int* __restrict__ supw, const int* __restrict__ cnt,
                                                   const int2* __restrict__ cvt, const int2* __restrict__ cee, int nv,
                                                   int ne, int* vofs, int* eofs) {
    if (supw[6]) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nv + ne; i += gridDim.x * blockDim.x) {
        const bool vt = i < nv;
        const int q = vt ? i : i - nv;
        const int2* list = vt ? cvt : cee;
        int lo = 0, hi = vt ? cnt[0] : cnt[1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (list[mid].x < q) lo = mid + 1;
            else hi = mid;
        }
        (vt ? vofs : eofs)[q] = lo;
    }
}

// One block: reduce the box partials; per family (0 = triangles, 1 = edges)
// the cell widths of the two grids.
__global__ void __launch_bounds__(256) k_grid(const int* __restrict__ gate, const float* __restrict__ bpart, int nblk, int nt, int ne,
                                              BpGrid* grid) {
    if (gated(gate)) return;
    __shared__ float red[4][BP_PART];
    // each thread folds whole partial records (BP_PART contiguous values),
    // then the wavefronts fold theirs with shuffles
    float w[BP_PART];
#pragma unroll
    for (int q = 0; q < BP_PART; ++q) w[q] = bp_identity(bp_op(q));
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < BP_PART; ++q) w[q] = bp_combine(bp_op(q), w[q], bpart[(size_t)b * BP_PART + q]);
    }
#pragma unroll
    for (int q = 0; q < BP_PART; ++q)
        for (int o = 32; o > 0; o >>= 1) w[q] = bp_combine(bp_op(q), w[q], __shfl_xor(w[q], o, 64));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < BP_PART; ++q) red[threadIdx.x >> 6][q] = w[q];
    }
    __syncthreads();
    if (threadIdx.x < BP_PART) {
        const int q = threadIdx.x, op = bp_op(q);
        red[0][q] = bp_combine(op, bp_combine(op, red[0][q], red[1][q]), bp_combine(op, red[2][q], red[3][q]));
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int f = threadIdx.x;
        const float* r = red[0] + f * BP_FAM;
        const double count = (double)max(1, f == 0 ? nt : ne);
        BpGrid g;
        g.ok = 1;
        g.use2 = 0;
        for (int c = 0; c < 3; ++c) {
            g.cs2[c] = (double)r[c] * CELL_MARGIN + 1e-30;
            g.cs1[c] = fmin(g.cs2[c], 3.0 * ((double)r[9 + c] / count) * CELL_MARGIN + 1e-30);
            double ext = (double)r[6 + c] - (double)r[3 + c];
            if (!isfinite(g.cs2[c]) || !isfinite(g.cs1[c]) || !isfinite(ext)) g.ok = 0;
            // targets wider than a grid-1 cell exist
            if ((double)r[c] * CELL_MARGIN > g.cs1[c]) g.use2 = 1;
        }
        grid[f] = g;
    }
}

// bucket counts of the targets' low-corner cells
__global__ void __launch_bounds__(256) k_cells(const int* __restrict__ gate, int m, const float* __restrict__ box, const BpGrid* __restrict__ gp,
                                               int* bucket_cnt, int P, int* overflow) {
    if (gated(gate)) return;
    const BpGrid g = *gp;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        int c[3], grid;
        if (!target_cell(box + 6 * (size_t)i, g, grid, c)) atomicOr(overflow, OVF_CELL);   // filed in cell 0
        atomicAdd(&bucket_cnt[cell_bucket(grid, c[0], c[1], c[2], P)], 1);
    }
}

// targets into their cell buckets as inline records (order inside a bucket
// is arbitrary: query outputs are sorted by target id)
__global__ void __launch_bounds__(256) k_bucket_fill(Dev d, int vt, int m, const float* __restrict__ box,
                                                     const BpGrid* __restrict__ gp, int P, int* cursor, BpRec* rec) {
    if (gated(d.gate)) return;
    const BpGrid g = *gp;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        int c[3], grid;
        target_cell(box + 6 * (size_t)i, g, grid, c);
        int pos = atomicAdd(&cursor[cell_bucket(grid, c[0], c[1], c[2], P)], 1);
        BpRec r;
        r.key = cell_key(grid, c[0], c[1], c[2]);
        r.id = i;
        if (vt) {
            TriRec tr = d.tri[i];
            r.a = tr.v0;
            r.b = tr.v1;
            r.c = tr.v2;
        } else {
            r.a = d.edges[2 * i];
            r.b = d.edges[2 * i + 1];
            r.c = -1;
        }
        for (int k = 0; k < 3; ++k) {
            r.lo[k] = box[6 * (size_t)i + k];
            r.hi[k] = box[6 * (size_t)i + 3 + k];
        }
        rec[pos] = r;
    }
}

// Query of one box against the cell buckets.  VT: query = vertex v,
// targets = triangles not incident to v; EE: query = edge e, targets = edges
// f > e sharing no vertex.  Three kernels, all built on group_query (G lanes
// per query):
//   k_query_count  counts each query's hits and keeps up to QK of them in
//                  `scratch`, sorted by target id;
//   k_query_copy   writes the queries whose hits fit the scratch to the
//                  candidate list at their offsets;
//   k_query_rescan finds the hits of the other (rare) queries again, one
//                  wavefront per query, and writes them sorted.
// Work and output per query are bounded (MAX_VISIT records, max_out pairs,
// at most 32 grid-1 and 8 grid-2 cells per axis and MAX_CELLS per grid,
// finite boxes only); hitting a bound sets the overflow flag and the step
// reports a capacity error instead of running away on a diverged state.
constexpr int MAX_VISIT = 1 << 16;
constexpr int MAX_CELLS = 4096;   // cells one query may visit in one grid
constexpr int MAX_HITS = 1024;    // largest per-query output bound (max_out)

// total of the last count + last offset -> n (clamped to cap), overflow flag
__global__ void k_count_total(const int* __restrict__ gate, const int* counts_scanned, const int* counts_raw, int m, int* n_out, int64_t cap,
                              int* overflow) {
    if (gated(gate)) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long tot = m > 0 ? (long long)counts_scanned[m - 1] + counts_raw[m - 1] : 0;
        overflow[PEAK_SLOT - 7] = max(overflow[PEAK_SLOT - 7], (int)min(tot, (long long)INT_MAX));
        if (tot > cap) {
            *overflow |= OVF_LIST;
            tot = cap;
        }
        *n_out = (int)tot;
    }
}

// Workgroups are dealt round-robin over the 8 XCDs; block b of a grid of
// nblk is given tile xcd_block(b, nblk), so that each XCD works through one
// contiguous range of tiles (a bijection of [0, nblk)).
__device__ __forceinline__ int xcd_block(int b, int nblk) {
    constexpr int X = 8;
    const int x = b % X, i = b / X;
    const int q = nblk / X, rem = nblk % X;
    return x * q + min(x, rem) + i;
}

// The hits of query q, found by the G lanes of a group (lane = this thread's
// place in it; the group is a G-aligned segment of a wavefront, `sub` its
// index there).  The lanes split the query's cells, lay the records of those
// cells' buckets end to end (prefix sum of the bucket lengths) and read them
// together, consecutive lanes on consecutive records; hits are compacted
// with a ballot and handed to hit(index, target id) in a fixed order (cells,
// then records).  Returns the hit count (capped at max_out + G); `full` is
// set when a bound is hit.
template <bool VT, int G, bool ET = false, typename Hit>
__device__ __forceinline__ int group_query(const Dev& d, int q, int lane, int sub, const float* __restrict__ qbox,
                                           const BpGrid& g, const int* __restrict__ bptr,
                                           const BpRec* __restrict__ rec, int P, int max_out, bool& full,
                                           Hit&& hit) {
    static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "lanes per query");
    const unsigned long long seg = G == 64 ? ~0ull : ((1ull << G) - 1);
    const float* qb = qbox + 6 * (size_t)q;
    const float ql[3] = {qb[0], qb[1], qb[2]}, qh[3] = {qb[3], qb[4], qb[5]};
    int qa = -1, qb2 = -1;
    if (!VT) {
        qa = d.edges[2 * q];
        qb2 = d.edges[2 * q + 1];
    }
    int cnt = 0, visits = 0;
    full = !(g.ok && isfinite(ql[0] + ql[1] + ql[2] + qh[0] + qh[1] + qh[2]));
    for (int grid = 0; grid < 1 + g.use2 && !full; ++grid) {
        const int span = grid ? 8 : 32;   // cells per axis a query may cover
        int lo[3], hi[3];
        if (!cell3g(ql, g, grid, lo) || !cell3g(qh, g, grid, hi)) {
            full = true;
            break;
        }
        for (int c = 0; c < 3; ++c) {
            lo[c] -= 1;
            if (hi[c] - lo[c] > span) full = true;
        }
        const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
        if (!full && nx * ny * nz > MAX_CELLS) full = true;
        if (full) break;
        const int ncell = nx * ny * nz;
        for (int c0 = 0; c0 < ncell && !full; c0 += G) {
            // this lane's cell and its bucket's record range
            const int c = c0 + lane;
            int s0 = 0, len = 0;
            long long key = 0;
            if (c < ncell) {
                const int cz = lo[2] + c % nz, cy = lo[1] + (c / nz) % ny, cx = lo[0] + c / (nz * ny);
                const unsigned b = cell_bucket(grid, cx, cy, cz, P);
                s0 = bptr[b];
                len = bptr[b + 1] - s0;
                key = cell_key(grid, cx, cy, cz);
            }
            int incl = len;
            for (int o = 1; o < G; o <<= 1) {
                const int t = __shfl_up(incl, o, G);
                if (lane >= o) incl += t;
            }
            const int V = __shfl(incl, G - 1, G);   // records of this chunk of cells
            const int excl = incl - len;
            visits += V;
            if (visits > MAX_VISIT) {
                full = true;
                break;
            }
            for (int t0 = 0; t0 < V; t0 += G) {
                // record t of the chunk: the cell j with excl_j <= t < excl_j + len_j
                // (the last lane whose exclusive prefix is <= t)
                const int t = min(t0 + lane, V - 1);
                int j = 0;
                for (int step = G / 2; step > 0; step >>= 1)
                    if (__shfl(excl, j + step, G) <= t) j += step;
                const int k = __shfl(s0, j, G) + (t - __shfl(excl, j, G));
                const long long kj = __shfl(key, j, G);
                bool pass = false;
                int id = 0;
                if (t0 + lane < V) {
                    const BpRec r = rec[k];
                    id = r.id;
                    pass = r.key == kj;
                    if (VT)
                        pass = pass && r.a != q && r.b != q && r.c != q;
                    else if (ET)   // edge query, triangle targets sharing no vertex with it
                        pass = pass && r.a != qa && r.a != qb2 && r.b != qa && r.b != qb2 && r.c != qa &&
                               r.c != qb2;
                    else
                        pass = pass && r.id > q && r.a != qa && r.a != qb2 && r.b != qa && r.b != qb2;
                    pass = pass && !(ql[0] > r.hi[0] || r.lo[0] > qh[0] || ql[1] > r.hi[1] || r.lo[1] > qh[1] ||
                                     ql[2] > r.hi[2] || r.lo[2] > qh[2]);
                }
                const unsigned long long gm = (__ballot(pass) >> (sub * G)) & seg;
                if (pass) hit(cnt + __popcll(gm & ((1ull << lane) - 1)), id);
                cnt += __popcll(gm);
            }
            if (cnt > max_out) full = true;
        }
    }
    return cnt;
}

// Counting pass: one group of G lanes per query.  The kept hits (at most
// QK) are ranked in LDS and written to the scratch sorted by target id.
// Blocks take consecutive queries and each XCD a contiguous range of blocks,
// so few queries are in flight per XCD and the records of their cells stay
// in its L2.
template <bool VT, int G>
__global__ void __launch_bounds__(256) k_query_count(Dev d, const float* __restrict__ qbox,
                                                     const BpGrid* __restrict__ gp, const int* __restrict__ bptr,
                                                     const BpRec* __restrict__ rec, int P, int* count, int* scratch,
                                                     int max_out, int* overflow, int* heavy_list, int* heavy_n) {
    if (gated(d.gate)) return;
    constexpr int GPB = 256 / G;
    __shared__ int res[GPB][QK];
    const int nq = VT ? d.nv : d.ne;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int sub = (threadIdx.x & 63) / G;
    const int q = xcd_block(blockIdx.x, gridDim.x) * GPB + grp;
    const BpGrid g = *gp;
    int cnt = 0;
    bool full = false;
    if (q < nq) {
        cnt = group_query<VT, G>(d, q, lane, sub, qbox, g, bptr, rec, P, max_out, full, [&](int idx, int id) {
            if (idx < QK) res[grp][idx] = id;
        });
        if (lane == 0) {
            count[q] = min(cnt, max_out);
            if (full) atomicOr(overflow, OVF_QUERY);
            // the queries whose hits do not fit the scratch, for k_query_rescan
            if (min(cnt, max_out) > QK) {
                const int h = atomicAdd(heavy_n, 1);
                if (h < nq) heavy_list[h] = q;
            }
        }
    }
    __syncthreads();
    // the kept hits in target-id order (ids are distinct within a query)
    if (q < nq && cnt <= QK) {
        int* sq = scratch + (size_t)q * QK;
        for (int i = lane; i < cnt; i += G) {
            const int v = res[grp][i];
            int rank = 0;
            for (int k2 = 0; k2 < cnt; ++k2) rank += res[grp][k2] < v;
            sq[rank] = v;
        }
    }
}

// Writing pass for the queries whose hits fit the scratch (at most QK): the
// G lanes of a query copy its sorted hits to the candidate list at its
// offset, consecutive lanes to consecutive entries.
template <int G>
__global__ void __launch_bounds__(256) k_query_copy(const int* __restrict__ gate, int nq, const int* __restrict__ ofs, const int* __restrict__ raw,
                                                    const int* __restrict__ scratch, int2* out, int64_t cap) {
    if (gated(gate)) return;
    constexpr int GPB = 256 / G;
    const int lane = threadIdx.x % G;
    const int q = xcd_block(blockIdx.x, gridDim.x) * GPB + threadIdx.x / G;
    if (q >= nq) return;
    const int k = raw[q], base = ofs[q];
    if (base < 0 || k > QK) return;
    const int* sq = scratch + (size_t)q * QK;
    for (int i = lane; i < k; i += G) {
        const int64_t pos = (int64_t)base + i;
        if (pos < cap) out[pos] = make_int2(q, sq[i]);
    }
}

// Writing pass for the queries with more than QK hits, listed by
// k_query_count (in no particular order: each one's output place is fixed by
// its offset).  The wavefronts of the whole grid take them one at a time, so
// that the heavy queries, which cluster where the cloth folds, are spread
// over every CU; a wavefront finds the query's hits again with group_query
// (G = 64) into LDS, ranks them and writes them sorted at the query's offset.
// The last workgroup out clears the list's count for the next pass.
template <bool VT>
__global__ void __launch_bounds__(256) k_query_rescan(Dev d, const float* __restrict__ qbox,
                                                      const BpGrid* __restrict__ gp, const int* __restrict__ bptr,
                                                      const BpRec* __restrict__ rec, int P,
                                                      const int* __restrict__ ofs, const int* __restrict__ raw,
                                                      int2* out, int64_t cap, int max_out, int* overflow,
                                                      const int* __restrict__ heavy_list, int* heavy_n) {
    if (gated(d.gate)) return;
    __shared__ int hits[4][MAX_HITS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const BpGrid g = *gp;
    const int nh = min(heavy_n[0], VT ? d.nv : d.ne);
    for (int h = blockIdx.x * 4 + w; h < nh; h += gridDim.x * 4) {
        const int qq = heavy_list[h];
        if (ofs[qq] < 0 || raw[qq] <= QK) continue;   // wavefront-uniform
        bool full = false;
        const int cnt = group_query<VT, 64>(d, qq, lane, 0, qbox, g, bptr, rec, P, max_out, full,
                                            [&](int idx, int id) {
                                                if (idx < MAX_HITS) hits[w][idx] = id;
                                            });
        if (full && lane == 0) atomicOr(overflow, OVF_QUERY);
        const int m = min(cnt, min(max_out, MAX_HITS));
        const int64_t base = ofs[qq];
        if (lane == 0 && base + m > cap) atomicOr(overflow, OVF_LIST);
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < m; i += 64) {
            const int v = hits[w][i];
            int rank = 0;
            for (int k2 = 0; k2 < m; ++k2) rank += hits[w][k2] < v;
            if (base + rank < cap) out[base + rank] = make_int2(qq, v);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&heavy_n[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&heavy_n[0], 0);
            atomicExch(&heavy_n[1], 0);
        }
    }
}

// ================================================================ TOI + merge
// For candidate i (VT in [0, n_vt), EE after): TOI and the keep flag
// TOI <= 1 (k_prev_match then adds the pairs of the previous constraint set
// and their life spans).  Work is taken in chunks of TOI_CHUNK candidates per block: every lane first
// settles the pairs that cannot hit (no root of the coplanarity cubic in
// [0, 1]); the rest go to an LDS queue that all lanes then drain, so the
// root refinement and the inside tests run on full wavefronts.
constexpr int TOI_CHUNK = 1024;
constexpr int TOI_FB = 32;        // fallback pairs per chunk taken by whole wavefronts
constexpr int TOI_LINE = 16;     // ints between the chunk counters (one 64-byte line each)

__device__ __forceinline__ void toi_finish(int i, bool vt, int nvt, double t, double* toi_vt, double* toi_ee,
                                           int* keep, int* cand_a, int do_merge) {
    if (vt) toi_vt[i] = t; else toi_ee[i - nvt] = t;
    if (!do_merge) return;
    // the pairs of the previous set that are still candidates are added,
    // with their life spans, by k_prev_match
    keep[i] = t <= 1.0 ? 1 : 0;
    cand_a[i] = 0;
}

__global__ void __launch_bounds__(256) k_toi_merge(Dev d, const float4* __restrict__ xm, const float4* __restrict__ xp,
                                                   const int2* __restrict__ cvt, const int2* __restrict__ cee,
                                                   int* cnt, double* toi_vt, double* toi_ee, int* keep,
                                                   int* cand_a, double* tpart, int do_merge, int* sched) {
    if (gated(d.gate)) return;
    __shared__ double wmin[4];
    __shared__ int queue[TOI_CHUNK + 256];   // pairs waiting for root refinement
    __shared__ int fbq[TOI_FB];   // pairs that need the sampled fallback
    __shared__ double fbe[TOI_FB];
    __shared__ int qn, fbn, s_ch;
    const int nvt = cnt[0], nee = cnt[1];
    const int total = nvt + nee;
    // next chunk of each XCD's range, one counter per 64-byte line (cleared
    // before the launch)
    int* next = sched;
    double tmin = NOHIT;
    // the chunks are split into 8 contiguous ranges, one per XCD (workgroups
    // are dealt round-robin over the XCDs), so that an XCD gathers the
    // positions of one region of the cloth, which then stay in its L2.
    // Workgroups claim chunks of their XCD's range one at a time and, once
    // it is used up, of the other ranges: the cost of a chunk varies (the
    // share of pairs that need root refinement, the rare sampled fallback),
    // and claiming keeps every CU busy until the last chunk is taken.
    const int nchunk = (total + TOI_CHUNK - 1) / TOI_CHUNK;
    const int per_x = (nchunk + 7) / 8;
    const int xcd = blockIdx.x % 8;
    int range = 0;   // thread 0 only: ranges already used up
    int q_left = 0;  // pairs still waiting in the queue
    for (;;) {
        if (threadIdx.x == 0) {
            int ch = -1;
            for (; range < 8; ++range) {
                const int x = (xcd + range) & 7;
                const int lim = min(nchunk, (x + 1) * per_x) - x * per_x;   // chunks of range x
                // a range seen used up is skipped without an atomic (the
                // counter only grows, so a stale read only costs the atomic)
                if (*(volatile int*)&next[TOI_LINE * x] >= lim) continue;
                const int c = atomicAdd(&next[TOI_LINE * x], 1);
                if (c < lim) {
                    ch = x * per_x + c;
                    break;
                }
            }
            s_ch = ch;
            qn = q_left;
            fbn = 0;
        }
        __syncthreads();
        const int ch = s_ch;
        const int base = ch * TOI_CHUNK;
        for (int k = threadIdx.x; ch >= 0 && k < TOI_CHUNK; k += blockDim.x) {
            const int i = base + k;
            if (i >= total) break;
            const bool vt = i < nvt;
            const int2 pr = vt ? cvt[i] : cee[i - nvt];
            d3 q0[4], q1[4];
            pair_points2(d, vt, pr.x, pr.y, xm, xp, q0, q1);
            if (pair_no_hit(vt, q0, q1))
                toi_finish(i, vt, nvt, NOHIT, toi_vt, toi_ee, keep, cand_a, do_merge);
            else
                queue[atomicAdd(&qn, 1)] = i;
        }
        __syncthreads();
        // root refinement in whole passes of the block: the queue is drained
        // down to fewer than 256 pairs, which wait for the next chunk's (all
        // of it after the last chunk), so that the lanes of a pass are busy
        const int nq = qn;
        const int take = ch < 0 ? nq : nq - nq % (int)blockDim.x;
        q_left = nq - take;
        for (int k = threadIdx.x; k < take; k += blockDim.x) {
            const int i = queue[q_left + k];
            const bool vt = i < nvt;
            const int2 pr = vt ? cvt[i] : cee[i - nvt];
            d3 q0[4], q1[4];
            pair_points2(d, vt, pr.x, pr.y, xm, xp, q0, q1);
            double eta = 0.0;
            double t = vt ? pair_toi_vt(q0, q1, eta) : pair_toi_ee(q0, q1, eta);
            if (eta > 0.0) {
                const int f = atomicAdd(&fbn, 1);
                if (f < TOI_FB) {
                    fbq[f] = i;
                    fbe[f] = eta;
                    continue;
                }
                t = vt ? sampled_toi<true>(q0, q1, eta) : sampled_toi<false>(q0, q1, eta);
            }
            tmin = fmin(tmin, t);
            toi_finish(i, vt, nvt, t, toi_vt, toi_ee, keep, cand_a, do_merge);
        }
        __syncthreads();
        // the sampled fallbacks (rare; a thousand distance evaluations each),
        // one pair per wavefront with the samples spread over its lanes
        const int nf = min(fbn, TOI_FB);
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int f = wave; f < nf; f += blockDim.x >> 6) {
            const int i = fbq[f];
            const bool vt = i < nvt;
            const int2 pr = vt ? cvt[i] : cee[i - nvt];
            d3 q0[4], q1[4];
            pair_points2(d, vt, pr.x, pr.y, xm, xp, q0, q1);
            const double t = vt ? sampled_toi_wave<true>(q0, q1, fbe[f], lane)
                                : sampled_toi_wave<false>(q0, q1, fbe[f], lane);
            tmin = fmin(tmin, t);
            if (lane == 0) toi_finish(i, vt, nvt, t, toi_vt, toi_ee, keep, cand_a, do_merge);
        }
        __syncthreads();   // the queues, their counts and s_ch are reused by the next chunk
        if (ch < 0) break;
    }
    tmin = warp_min(tmin);
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = tmin;
    __syncthreads();
    if (threadIdx.x == 0) tpart[blockIdx.x] = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
}

// Second half of the constraint-set update, C_o = {TOI <= 1} U (C_{o-1}
// intersected with the candidates): each pair of the previous set looks
// itself up among the candidates of its query (the candidate list is grouped
// by query at the offsets ofs and sorted by target inside a group) and, when
// found, keeps that candidate and hands it its life span.  Runs after
// k_toi_merge, which set keep = (TOI <= 1) and a = 0 for every candidate.
__global__ void __launch_bounds__(256) k_prev_match(const int* __restrict__ gate, const int* __restrict__ cnt, const int2* __restrict__ prev,
                                                    const int* __restrict__ prev_a, const int2* __restrict__ cvt,
                                                    const int2* __restrict__ cee, const int* __restrict__ vofs,
                                                    const int* __restrict__ eofs, int nv, int ne, int* keep,
                                                    int* cand_a) {
    if (gated(gate)) return;
    const int nvt = cnt[0], nee = cnt[1], pvt = cnt[4], pee = cnt[5];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < pvt + pee; p += gridDim.x * blockDim.x) {
        const bool vt = p < pvt;
        const int2 pr = prev[p];
        const int nq = vt ? nv : ne, nl = vt ? nvt : nee;
        if (pr.x < 0 || pr.x >= nq) continue;
        const int* ofs = vt ? vofs : eofs;
        const int2* list = vt ? cvt : cee;
        int lo = min(ofs[pr.x], nl);
        const int end = pr.x + 1 < nq ? min(ofs[pr.x + 1], nl) : nl;
        int hi = end;
        while (lo < hi) {   // first candidate of the query with target >= pr.y
            const int mid = (lo + hi) >> 1;
            if (list[mid].y < pr.y) lo = mid + 1;
            else hi = mid;
        }
        if (lo < end && list[lo].x == pr.x && list[lo].y == pr.y) {
            const int i = (vt ? 0 : nvt) + lo;
            keep[i] = 1;
            cand_a[i] = prev_a[p];
        }
    }
}

// obstacles: TOI on (xm, xp) and membership with carried life spans
__global__ void __launch_bounds__(256) k_obstacles_outer(Dev d, const float* __restrict__ xm, const float* __restrict__ xp,
                                  double* tpart, int* n_ob) {
    if (gated(d.gate)) return;
    __shared__ double wmin[4];
    const int nob = d.nob;
    const ObstD* ob = d.ob;
    int* ob_a = d.ob_a;
    const double dhat = d.dhat;
    int members = 0;
    const int n = d.nv;
    double tmin = NOHIT;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        d3 a = ld3(xm, n, v), b = ld3(xp, n, v);
        for (int j = 0; j < nob; ++j) {
            double t = obst_toi(ob[j], a, b);
            tmin = fmin(tmin, t);
            d3 rv;
            double rad;
            double pm = obst_phi(ob[j], a, rv, rad), pp = obst_phi(ob[j], b, rv, rad);
            bool mem = !d.pinned[v] && (t <= 1.0 || pm < dhat || pp < dhat);
            int prev = ob_a[(size_t)j * n + v];
            ob_a[(size_t)j * n + v] = mem ? (prev >= 0 ? prev : 0) : -1;
            members += mem;
        }
    }
    if (members) atomicAdd(n_ob, members);
    tmin = warp_min(tmin);
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = tmin;
    __syncthreads();
    if (threadIdx.x == 0) tpart[blockIdx.x] = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
}

// Stage t_TOI = minimum of the per-block partials of the TOI and obstacle
// kernels (npart of them) and tmin_bits[0]; s = 1 (no hit) or alpha t_TOI;
// running minimum for the statistics and the stage's own t_TOI (the exiting
// one after the last stage).  One block of 256 threads.
__global__ void k_step_length(const int* __restrict__ gate, const double* __restrict__ tpart, int npart, unsigned long long* tmin_bits,
                              double alpha, double* s_dev, const int* __restrict__ fail) {
    if (gated(gate)) return;
    __shared__ double red[256];
    double m = NOHIT;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) m = fmin(m, tpart[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double t = fmin(red[0], __longlong_as_double((long long)tmin_bits[0]));
        tmin_bits[0] = (unsigned long long)__double_as_longlong(t);
        // a stage whose candidate or constraint lists overflowed has pairs
        // without a time of impact: the block does not move (the step is
        // rolled back at its end and reports the overflow)
        s_dev[0] = (fail && (*fail & (OVF_QUERY | OVF_CELL | OVF_LIST | OVF_CONS))) ? 0.0 : (t > 1.0 ? 1.0 : alpha * t);
        tmin_bits[2] = tmin_bits[0];
        if (tmin_bits[0] < tmin_bits[1]) tmin_bits[1] = tmin_bits[0];
        tmin_bits[0] = (unsigned long long)__double_as_longlong(NOHIT);
    }
}

// compaction of kept candidates into the new constraint list (order kept)
__global__ void k_compact(const int* __restrict__ gate, const int2* __restrict__ cvt, const int2* __restrict__ cee, int* cnt,
                          const int* __restrict__ keep, const int* __restrict__ ofs, const int* __restrict__ cand_a,
                          int2* cpair, int* ca, int64_t ccap) {
    if (gated(gate)) return;
    const int nvt = cnt[0], nee = cnt[1];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nvt + nee; i += gridDim.x * blockDim.x) {
        if (keep[i]) {
            int o = ofs[i];
            if (o < ccap) {
                cpair[o] = i < nvt ? cvt[i] : cee[i - nvt];
                ca[o] = cand_a[i];
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int tot = nvt + nee;
        int nk = tot > 0 ? ofs[tot - 1] + keep[tot - 1] : 0;
        int nk_vt = nvt > 0 ? (nvt < tot ? ofs[nvt] : nk) : 0;
        if (nk > ccap) {   // the set is cut to the capacity and the step reports it
            cnt[7] |= OVF_CONS;
            nk = (int)ccap;
            nk_vt = min(nk_vt, nk);
        }
        cnt[2] = nk_vt;
        cnt[3] = nk - nk_vt;
    }
}

// ================================================================ frozen data
// Closest-point parameters and normals at x- (start of the block).
__global__ void __launch_bounds__(256) k_freeze(Dev d, const int* cnt, const int2* __restrict__ cpair, double2* clam, float4* cnrm) {
    if (gated(d.gate)) return;
    const int nvt = cnt[2], nc = cnt[2] + cnt[3];
    const int n = d.nv;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        int2 pr = cpair[p];
        d3 q[4];
        pair_points(d, p < nvt, pr.x, pr.y, d.xm, q);
        double l1, l2;
        d3 nn;
        if (p < nvt) {
            tri_closest(q[0], q[1], q[2], q[3], l1, l2);
            nn = cross(q[2] - q[1], q[3] - q[1]);
            double nl = sqrt(dot(nn, nn));
            nn = nl > 0 ? nn * (1.0 / nl) : mk(0, 1, 0);
            if (dot(nn, q[0] - q[1]) < 0) nn = nn * -1.0;
        } else {
            seg_closest(q[0], q[1], q[2], q[3], l1, l2);
            d3 dd = lerp(q[2], q[3], l2) - lerp(q[0], q[1], l1);
            double dl = sqrt(dot(dd, dd));
            if (dl > 0) {
                nn = dd * (1.0 / dl);
            } else {
                nn = cross(q[1] - q[0], q[3] - q[2]);
                double nl = sqrt(dot(nn, nn));
                nn = nl > 0 ? nn * (1.0 / nl) : mk(0, 1, 0);
            }
        }
        clam[p] = make_double2(l1, l2);
        cnrm[p] = make_float4((float)nn.x, (float)nn.y, (float)nn.z, 0.f);
        (void)n;
    }
}

// vertex -> slot incidence (slot = 4 * constraint + corner)
__global__ void k_slot_count(Dev d, const int* cnt, const int2* __restrict__ cpair, int* vcnt) {
    if (gated(d.gate)) return;
    const int nvt = cnt[2], nc = cnt[2] + cnt[3];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        int2 pr = cpair[p];
        int id[4];
        pair_ids(d, p < nvt, pr.x, pr.y, id);
        for (int k = 0; k < 4; ++k) atomicAdd(&vcnt[id[k]], 1);
    }
}

__global__ void k_slot_fill(Dev d, const int* cnt, const int2* __restrict__ cpair, int* cursor, int* vslot) {
    if (gated(d.gate)) return;
    const int nvt = cnt[2], nc = cnt[2] + cnt[3];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x) {
        int2 pr = cpair[p];
        int id[4];
        pair_ids(d, p < nvt, pr.x, pr.y, id);
        for (int k = 0; k < 4; ++k) vslot[atomicAdd(&cursor[id[k]], 1)] = 4 * p + k;
    }
}

// sort each vertex's slots (deterministic accumulation order) and flag
// contact vertices (in a pair constraint or an obstacle constraint)
__global__ void __launch_bounds__(256) k_slot_sort(Dev d, const int* __restrict__ ptr, int* vslot, const int* __restrict__ ob_a, int nob,
                            int* flag) {
    if (gated(d.gate)) return;
    const int n = d.nv;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int b0 = ptr[v], b1 = ptr[v + 1];
        for (int i = b0 + 1; i < b1; ++i) {
            int key = vslot[i], j = i - 1;
            while (j >= b0 && vslot[j] > key) {
                vslot[j + 1] = vslot[j];
                --j;
            }
            vslot[j + 1] = key;
        }
        bool f = b1 > b0;
        for (int j = 0; j < nob; ++j) f |= ob_a[(size_t)j * n + v] >= 0;
        flag[v] = (f && !d.pinned[v]) ? 1 : 0;
    }
}

__global__ void k_cv_compact(const int* __restrict__ gate, int n, const int* __restrict__ flag, const int* __restrict__ ofs, int* list, int* n_out,
                             int* wchg) {
    if (gated(gate)) return;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (flag[v]) list[ofs[v]] = v;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_out = n > 0 ? ofs[n - 1] + flag[n - 1] : 0;
        *wchg = 1;   // a new constraint set: refactor
    }
}

// ================================================================ per iteration
// Targets of the pair constraints at x^k, stored per slot as (w, w (y - x)):
// half-space projection with the
// frozen normal and closest-point parameters (minimum-norm correction over
// movable vertices), weight w = k * 2^a (Eq. (exp) with K = 2; other K use powf).
// the four slots of pair constraint p (VT when vt) with life span a, from
// the positions X
__device__ __forceinline__ void pair_target(const Dev& d, int p, bool vt, int2 pr, const float* __restrict__ X,
                                            const double2* __restrict__ clam, const float4* __restrict__ cnrm,
                                            int a, float kc, float Kb, float dhat, float4* slot) {
    const int n = d.nv;
    {
        int id[4];
        pair_ids(d, vt, pr.x, pr.y, id);
        float l1 = (float)clam[p].x, l2 = (float)clam[p].y;
        float c[4];
        if (vt) {
            c[0] = 1.f; c[1] = -(1.f - l1 - l2); c[2] = -l1; c[3] = -l2;
        } else {
            c[0] = -(1.f - l1); c[1] = -l1; c[2] = 1.f - l2; c[3] = l2;
        }
        float4 nr = cnrm[p];
        float gx = -dhat, den = 0.f;
        float xs[4][3];
        float cm[4];
        for (int k = 0; k < 4; ++k) {
            xs[k][0] = X[id[k]]; xs[k][1] = X[n + id[k]]; xs[k][2] = X[2 * n + id[k]];
            gx += c[k] * (nr.x * xs[k][0] + nr.y * xs[k][1] + nr.z * xs[k][2]);
            cm[k] = d.pinned[id[k]] ? 0.f : c[k];
            den += cm[k] * cm[k];
        }
        float delta = (gx < 0.f && den > 0.f) ? -gx / den : 0.f;
        float w = (Kb == 2.0f) ? ldexpf(kc, a) : kc * powf(Kb, (float)a);
        for (int k = 0; k < 4; ++k) {   // (w, w (y - x)) with y - x = c_k delta n
            float s = cm[k] * delta;
            slot[4 * (size_t)p + k] = make_float4(w, w * s * nr.x, w * s * nr.y, w * s * nr.z);
        }
    }
}

__global__ void __launch_bounds__(256) k_pair_targets(Dev d, const int* cnt, const int2* __restrict__ cpair, const int* __restrict__ ca,
                               const double2* __restrict__ clam, const float4* __restrict__ cnrm, float kc, float Kb,
                               float dhat, float4* slot, int force_k) {
    if (gated(d.gate)) return;
    const int nvt = cnt[2], nc = cnt[2] + cnt[3];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += gridDim.x * blockDim.x)
        pair_target(d, p, p < nvt, cpair[p], d.xk, clam, cnrm, force_k ? 0 : ca[p], kc, Kb, dhat, slot);
}

// Q(lambda) of Eq. (query) at one sample of a pair with corners q0 (x-) and
// q1 (the iterate): VT, vertex 0 against the point of triangle (1, 2, 3) at
// barycentrics (l1, l2); EE, edge (0, 1) at l1 against edge (2, 3) at l2.
__device__ __forceinline__ double pair_query(bool vt, const d3* q0, const d3* q1, double l1, double l2) {
    d3 a0, a1;
    if (vt) {
        d3 p20 = q0[1] + (q0[2] - q0[1]) * l1 + (q0[3] - q0[1]) * l2;
        d3 p21 = q1[1] + (q1[2] - q1[1]) * l1 + (q1[3] - q1[1]) * l2;
        a0 = p20 - q0[0];
        a1 = p21 - q1[0];
    } else {
        a0 = (q0[2] + (q0[3] - q0[2]) * l2) - (q0[0] + (q0[1] - q0[0]) * l1);
        a1 = (q1[2] + (q1[3] - q1[2]) * l2) - (q1[0] + (q1[1] - q1[0]) * l1);
    }
    return dot(a1, a0);
}

constexpr int ADAPT_M0 = 2, ADAPT_MMAX = 8;

// Adaptive density (end of section 4.1): the change ratio of rho* (Eq.
// (sample_bound)) over the iteration, with rho* proportional to
// H0^2 / (L (H1 + 2 L)), L the longest primitive edge and H1 the largest
// distance between a point of one primitive and one of the other over the
// motion (both convex in time, so the larger end value), against their
// values at x- alone; then the refined level min(MMAX, floor(M0 / ratio)).
__device__ __forceinline__ int adaptive_level(bool vt, const d3* q0, const d3* q1) {
    auto len = [](d3 a) { return sqrt(dot(a, a)); };
    double L0, L1, H0, H1;
    if (vt) {
        L0 = fmax(fmax(len(q0[1] - q0[2]), len(q0[2] - q0[3])), len(q0[3] - q0[1]));
        L1 = fmax(L0, fmax(fmax(len(q1[1] - q1[2]), len(q1[2] - q1[3])), len(q1[3] - q1[1])));
        H0 = fmax(fmax(len(q0[0] - q0[1]), len(q0[0] - q0[2])), len(q0[0] - q0[3]));
        H1 = fmax(H0, fmax(fmax(len(q1[0] - q1[1]), len(q1[0] - q1[2])), len(q1[0] - q1[3])));
    } else {
        L0 = fmax(len(q0[0] - q0[1]), len(q0[2] - q0[3]));
        L1 = fmax(L0, fmax(len(q1[0] - q1[1]), len(q1[2] - q1[3])));
        H0 = fmax(fmax(len(q0[0] - q0[2]), len(q0[0] - q0[3])), fmax(len(q0[1] - q0[2]), len(q0[1] - q0[3])));
        H1 = fmax(H0, fmax(fmax(len(q1[0] - q1[2]), len(q1[0] - q1[3])),
                           fmax(len(q1[1] - q1[2]), len(q1[1] - q1[3]))));
    }
    const double ratio = (L0 * (H0 + 2.0 * L0)) / (L1 * (H1 + 2.0 * L1));
    const double m = floor((double)ADAPT_M0 / ratio);
    return m >= (double)ADAPT_MMAX ? ADAPT_MMAX : (int)m;
}

// Partial CCD on (x-, x^{k+1}): active when Q(lambda) <= 0 at a sample
// (three fixed samples plus the frozen closest point; with `adapt`, pairs
// whose rho* shrank use the refined set of their level instead of the
// fixed samples: the centroids of the m^2 sub-triangles of the barycentric
// triangle (VT) or the centres of the m x m cells of the parameter square
// (EE)); a <- active ? min(a+1, a_max) : 0.  Obstacles: active when
// phi(x^{k+1}) < d_hat.
// With `tg`, the pair constraints' targets of the next iteration follow at
// once (what k_pair_targets would compute from the new life spans and
// xnew, which is the next iteration's x^k).
__global__ void __launch_bounds__(256) k_partial_ccd(Dev d, const int* cnt, const int2* __restrict__ cpair, int* ca,
                              const double2* __restrict__ clam, int amax, const float* __restrict__ xnew,
                              int* wchg, int adapt, int tg, const float4* __restrict__ cnrm, float kc,
                              float Kb, float dhat_f, float4* slot) {
    if (gated(d.gate)) return;
    bool changed = false;
    const int nob = d.nob;
    const ObstD* ob = d.ob;
    int* ob_a = d.ob_a;
    const double dhat = d.dhat;
    const int nvt = cnt[2], nc = cnt[2] + cnt[3];
    const int n = d.nv;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nc + n; p += gridDim.x * blockDim.x) {
        if (p < nc) {
            int2 pr = cpair[p];
            bool vt = p < nvt;
            d3 q0[4], q1[4];
            pair_points(d, vt, pr.x, pr.y, d.xm, q0);
            pair_points(d, vt, pr.x, pr.y, xnew, q1);
            bool act = false;
            const double2 lf = clam[p];
            const int m = adapt ? adaptive_level(vt, q0, q1) : ADAPT_M0;
            if (m <= ADAPT_M0) {
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    // samples: VT barycentrics (1/6, 1/6), (2/3, 1/6), (1/6, 2/3);
                    // EE parameters (1/4, 1/4), (1/2, 1/2), (3/4, 3/4)
                    double l1, l2;
                    if (s == 0) {
                        l1 = vt ? 1.0 / 6 : 0.25;
                        l2 = vt ? 1.0 / 6 : 0.25;
                    } else if (s == 1) {
                        l1 = vt ? 2.0 / 3 : 0.5;
                        l2 = vt ? 1.0 / 6 : 0.5;
                    } else {
                        l1 = vt ? 1.0 / 6 : 0.75;
                        l2 = vt ? 2.0 / 3 : 0.75;
                    }
                    act |= pair_query(vt, q0, q1, l1, l2) <= 0.0;
                }
            } else if (vt) {
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m - i; ++j) {
                        act |= pair_query(vt, q0, q1, (i + 1.0 / 3) / m, (j + 1.0 / 3) / m) <= 0.0;
                        if (i + j <= m - 2) act |= pair_query(vt, q0, q1, (i + 2.0 / 3) / m, (j + 2.0 / 3) / m) <= 0.0;
                    }
            } else {
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j) act |= pair_query(vt, q0, q1, (i + 0.5) / m, (j + 0.5) / m) <= 0.0;
            }
            // the frozen closest point is always a sample
            act |= pair_query(vt, q0, q1, lf.x, lf.y) <= 0.0;
            const int a = ca[p], na = act ? min(a + 1, amax) : 0;
            ca[p] = na;
            changed |= na != a;
            if (tg) pair_target(d, p, vt, pr, xnew, clam, cnrm, na, kc, Kb, dhat_f, slot);
        } else {
            int v = p - nc;
            d3 x = ld3(xnew, n, v);
            for (int j = 0; j < nob; ++j) {
                int a = ob_a[(size_t)j * n + v];
                if (a < 0) continue;
                d3 rv;
                double rad;
                bool act = obst_phi(ob[j], x, rv, rad) < dhat;
                const int na = act ? min(a + 1, amax) : 0;
                ob_a[(size_t)j * n + v] = na;
                changed |= na != a;
            }
        }
    }
    if (__ballot(changed) && (threadIdx.x & 63) == 0) *wchg = 1;
}

// Eight consecutive basis entries of a row (16 bytes of BF16 or 32 of FP32)
template <typename UT>
struct RowChunkG;
template <>
struct RowChunkG<uint16_t> {
    uint4 a;
    __device__ __forceinline__ void load(const uint16_t* __restrict__ U, size_t off) {
        a = *reinterpret_cast<const uint4*>(U + off);
    }
    __device__ __forceinline__ void unpack(float u[8]) const {
        u[0] = __uint_as_float(a.x << 16); u[1] = __uint_as_float(a.x & 0xffff0000u);
        u[2] = __uint_as_float(a.y << 16); u[3] = __uint_as_float(a.y & 0xffff0000u);
        u[4] = __uint_as_float(a.z << 16); u[5] = __uint_as_float(a.z & 0xffff0000u);
        u[6] = __uint_as_float(a.w << 16); u[7] = __uint_as_float(a.w & 0xffff0000u);
    }
};
template <>
struct RowChunkG<float> {
    float4 a, b;
    __device__ __forceinline__ void load(const float* __restrict__ U, size_t off) {
        const float4* p = reinterpret_cast<const float4*>(U + off);
        a = p[0];
        b = p[1];
    }
    __device__ __forceinline__ void unpack(float u[8]) const {
        u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
        u[4] = b.x; u[5] = b.y; u[6] = b.z; u[7] = b.w;
    }
};

constexpr int GRAM_MIN_PER_CHUNK = 32;
__device__ __forceinline__ int gram_per_chunk(int ncv, int nchunk) {
    return max(GRAM_MIN_PER_CHUNK, (ncv + nchunk - 1) / nchunk);
}

// Gram of the contact rows, Eq. (uu): sum over contact vertices j of
// W_j U_j U_j^T (r x r, FP64 partial per chunk of vertices), on the matrix
// cores: the upper block triangle of 16 x 16 tiles (r padded to a multiple
// of 16 with zero columns) is dealt to the four wavefronts of a block,
// GRAM_TW tiles each (blockIdx.y picks a group of 4 GRAM_TW tiles,
// blockIdx.x a chunk of the contact-vertex list), and each
// v_mfma_f64_16x16x4f64 adds four vertices to one tile: lane l supplies
// W u(row l % 16) and u(column l % 16) of vertex l / 16 and holds rows
// l / 16 + 4 e (e = 0..3) of column l % 16 of the tile.  Vertices are staged 32
// at a time in LDS as W-scaled (FP64) and plain (FP32) rows.
constexpr int GRAM_TW = 10;   // 16 x 16 FP64 tiles per wavefront
// Collision weight W_v of a contact vertex (a row of the Gram), summed as the
// local step sums it (pair slots in slot order, then obstacles), so that the
// contact matrix can be formed while the local step runs.
__device__ __forceinline__ float contact_weight(const Dev& d, int v, int force_k) {
    float Wv = 0.f;
    for (int j = d.vslot_ptr[v], e = d.vslot_ptr[v + 1]; j < e; ++j) Wv += d.slot[d.vslot[j]].x;
    for (int j = 0; j < d.nob; ++j) {
        int a = d.ob_a[j * d.nv + v];
        if (a < 0) continue;
        if (force_k) a = 0;
        const float w = (d.Kb == 2.0f) ? ldexpf(d.kc, a) : d.kc * powf(d.Kb, (float)a);
        Wv += w;
        if (d.mu > 0.0f) {
            // the friction weight, from the same iterate as the local step
            const int n = d.nv;
            const float x0 = d.xk[v], x1 = d.xk[n + v], x2 = d.xk[2 * n + v];
            const ObstD& o = d.ob[j];
            double ox, oy, oz;
            const double rad = obstacle_radial(o, x0, x1, x2, ox, oy, oz);
            double ux, uy, uz;
            Wv += (float)obstacle_friction(d, o, w, ox, oy, oz, rad, x0, x1, x2, d.xstar[v], d.xstar[n + v],
                                           d.xstar[2 * n + v], ux, uy, uz);
        }
    }
    return Wv;
}

typedef double gram_d4 __attribute__((ext_vector_type(4)));
template <typename UT>
__global__ void __launch_bounds__(256) k_gram(Dev d, const int* __restrict__ cvlist, const int* __restrict__ n_cv,
                                            int nchunk, double* part, const int* __restrict__ wchg, int force_k) {
    if (gated(d.gate) || !*wchg) return;   // no weight changed: the last factorization stands
    constexpr int VB = 32;   // contact vertices staged per round (a multiple of 4)
    __shared__ float us[VB][MAX_R];
    __shared__ double ws[VB][MAX_R];
    __shared__ int vidx[VB];
    __shared__ float wv[VB];
    const int r = d.r;
    const int R16 = (r + 15) >> 4;   // tile rows
    const int ncv = *n_cv;
    const int per = gram_per_chunk(ncv, nchunk);
    const int c0 = blockIdx.x * per, c1 = min(ncv, c0 + per);
    if (c0 >= c1) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, kv = lane >> 4;   // operand row / column, vertex of the four
    // this wavefront's tiles t = (blockIdx.y GRAM_TW + s) 4 + wave -> (ti, tj),
    // ti <= tj, row-major over the upper block triangle (wave-uniform)
    int ti[GRAM_TW], tj[GRAM_TW];
    bool on[GRAM_TW];
#pragma unroll
    for (int s = 0; s < GRAM_TW; ++s) {
        const int t = (blockIdx.y * GRAM_TW + s) * 4 + wave;
        on[s] = t < R16 * (R16 + 1) / 2;
        int a = 0, rem = on[s] ? t : 0;
        while (rem >= R16 - a) {
            rem -= R16 - a;
            ++a;
        }
        ti[s] = a;
        tj[s] = a + rem;
    }
    // FP64 products and sums: the weights span many orders of magnitude
    // (k 2^a), and an FP32 Gram's rounding reaches the scale of Lambda~'s
    // smallest eigenvalues, which can cost A its definiteness
    gram_d4 acc[GRAM_TW];
#pragma unroll
    for (int s = 0; s < GRAM_TW; ++s) acc[s] = gram_d4{0.0, 0.0, 0.0, 0.0};
    const UT* U = static_cast<const UT*>(d.U);
    const int ncg = r >> 3;            // groups of 8 basis columns per row
    const int ncg16 = R16 * 2;         // the same, up to the padded width
    for (int base = c0; base < c1; base += VB) {
        const int m = min(VB, c1 - base);
        __syncthreads();
        // the round's vertices and weights first, then every row's 8-column
        // groups with one wide load each, all independent of each other
        if (threadIdx.x < VB) {
            const int v = threadIdx.x < m ? cvlist[base + threadIdx.x] : -1;
            vidx[threadIdx.x] = v;
            wv[threadIdx.x] = v >= 0 ? contact_weight(d, v, force_k) : 0.f;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < VB * ncg16; q += 256) {
            const int vv = q / ncg16, cg = q % ncg16;
            const int v = vidx[vv];
            float u[8];
            if (v >= 0 && cg < ncg) {
                RowChunkG<UT> rc;
                rc.load(U, (size_t)v * r + cg * 8);
                rc.unpack(u);
            } else {
                for (int k = 0; k < 8; ++k) u[k] = 0.f;
            }
            const double w = (double)wv[vv];
            for (int k = 0; k < 8; ++k) {
                us[vv][cg * 8 + k] = u[k];
                ws[vv][cg * 8 + k] = w * (double)u[k];   // exact
            }
        }
        __syncthreads();
        for (int v0 = 0; v0 < m; v0 += 4) {
#pragma unroll
            for (int s = 0; s < GRAM_TW; ++s)
                if (on[s]) {
                    const double a = ws[v0 + kv][ti[s] * 16 + row];
                    const double b = (double)us[v0 + kv][tj[s] * 16 + row];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
        }
    }
#pragma unroll
    for (int s = 0; s < GRAM_TW; ++s) {
        if (!on[s]) continue;
        const int col = tj[s] * 16 + row;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int rw = ti[s] * 16 + kv + 4 * e;
            if (rw < r && col < r) part[((size_t)blockIdx.x * r + rw) * r + col] = acc[s][e];
        }
    }
}

// Packed lower triangle, column-major: column k holds rows k..r-1 at
// pk_off(k) = k r - k (k - 1) / 2, so that every column is contiguous.
__device__ __forceinline__ int pk_off(int k, int r) { return k * r - (k * (k - 1)) / 2; }
__device__ __forceinline__ void pk_entry(int e, int r, int& i, int& k) {
    // largest k with pk_off(k) <= e (pk_off is increasing in k)
    double b = 2.0 * r + 1.0;
    int kk = (int)((b - sqrt(b * b - 8.0 * e)) * 0.5);
    kk = max(0, min(r - 1, kk));
    while (kk > 0 && pk_off(kk, r) > e) --kk;
    while (kk + 1 < r && pk_off(kk + 1, r) <= e) ++kk;
    k = kk;
    i = k + (e - pk_off(k, r));
}

// First level of A = Lambda~ + sum of the Gram chunks: block (entry tile,
// group g) sums the chunks of group g for its entries in FP64.  The chunk
// partials hold the upper block triangle: A(i, k) = part(k, i) for k <= i.
constexpr int GRAM_GROUPS = GRAM_GROUPS_MAX;
__global__ void __launch_bounds__(256) k_gram_reduce(Dev d, const double* __restrict__ part, int nchunk,
                                                     const int* __restrict__ n_cv, double* __restrict__ gred,
                                                     const int* __restrict__ wchg) {
    if (gated(d.gate) || !*wchg) return;
    const int r = d.r;
    const int ncv = *n_cv;
    if (ncv == 0) return;
    const int per = gram_per_chunk(ncv, nchunk);
    const int used = min(nchunk, (ncv + per - 1) / per);
    const int tot = r * (r + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int g = blockIdx.y;
    const int per_g = (used + GRAM_GROUPS - 1) / GRAM_GROUPS;
    const int c0 = g * per_g, c1 = min(used, c0 + per_g);
    int i, k;
    pk_entry(e, r, i, k);
    double acc = 0.0;
#pragma unroll 4
    for (int c = c0; c < c1; ++c) acc += part[((size_t)c * r + k) * r + i];
    gred[(size_t)g * tot + e] = acc;
}

// packed lower triangle, row-major: A(i, j), j <= i, at i (i + 1) / 2 + j
__device__ __forceinline__ int rm(int i, int j) { return i * (i + 1) / 2 + j; }
__device__ __forceinline__ void tri_rc(int e, int& i, int& j) {
    i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    while (i * (i + 1) / 2 > e) --i;
    j = e - i * (i + 1) / 2;
}

// A = Lambda~ + the group sums, packed row-major (second reduction level).
__global__ void __launch_bounds__(256) k_gram_final(Dev d, const double* __restrict__ gred,
                                                    const int* __restrict__ n_cv, double* __restrict__ Arm,
                                                    const int* __restrict__ wchg) {
    if (gated(d.gate) || !*wchg) return;
    if (*n_cv == 0) return;
    const int r = d.r;
    const int tot = r * (r + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    int i, k;
    tri_rc(e, i, k);
    const int ec = pk_off(k, r) + (i - k);   // the same entry in the column-major group sums
    double s = d.Lam[(size_t)i * r + k];
    for (int g = 0; g < GRAM_GROUPS; ++g) s += gred[(size_t)g * tot + ec];
    Arm[e] = s;
}

// Eq. (uu), precomputed form: the upper triangle of U_j U_j^T of every
// vertex, entry e of vertex v at UU[v tot + e] in the packed column-major
// order of the group sums (pk_off), from the stored basis values (exact in
// FP32 for a BF16 basis).  Block = vertex, threads over the entries.
__device__ __forceinline__ float uu_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float uu_val(float f) { return f; }

template <typename UT>
__global__ void __launch_bounds__(256) k_uu_build(Dev d, float* __restrict__ UU) {
    __shared__ float u[MAX_R];
    const int r = d.r;
    const int tot = r * (r + 1) / 2;
    const UT* __restrict__ U = static_cast<const UT*>(d.U);
    for (int v = blockIdx.x; v < d.nv; v += gridDim.x) {
        for (int a = threadIdx.x; a < r; a += blockDim.x) u[a] = uu_val(U[(size_t)v * r + a]);
        __syncthreads();
        float* out = UU + (size_t)v * tot;
        for (int k = 0; k < r; ++k) {
            const float uk = u[k];
            const int o = pk_off(k, r) - k;
            for (int i = k + threadIdx.x; i < r; i += blockDim.x) out[o + i] = u[i] * uk;
        }
        __syncthreads();
    }
}

// Group sums of the contact part of A from the store: block (entry tile,
// group g) sums W_j UU_j over group g's share of the contact-vertex list in
// FP64, the weights of a round of 64 vertices staged in LDS (summed as the
// local step sums them), and writes the layout k_gram_reduce writes.
__global__ void __launch_bounds__(256) k_uu_sum(Dev d, const int* __restrict__ cvlist,
                                                const int* __restrict__ n_cv, double* __restrict__ gred,
                                                const int* __restrict__ wchg, int force_k) {
    if (gated(d.gate) || !*wchg) return;
    const int ncv = *n_cv;
    if (ncv == 0) return;
    const int r = d.r;
    const int tot = r * (r + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    const int per_g = (ncv + gridDim.y - 1) / gridDim.y;
    const int j0 = g * per_g, j1 = min(ncv, j0 + per_g);
    __shared__ float ws[64];
    __shared__ int vs[64];
    double acc = 0.0;
    for (int jb = j0; jb < j1; jb += 64) {
        const int m = min(64, j1 - jb);
        if (threadIdx.x < m) {
            const int v = cvlist[jb + threadIdx.x];
            vs[threadIdx.x] = v;
            ws[threadIdx.x] = contact_weight(d, v, force_k);
        }
        __syncthreads();
        if (e < tot)
            for (int t = 0; t < m; ++t) acc += (double)ws[t] * (double)d.UU[(size_t)vs[t] * tot + e];
        __syncthreads();
    }
    if (e < tot) gred[(size_t)g * tot + e] = acc;
}


constexpr int CHOL_PANEL = 16;

__device__ __forceinline__ double bcast_f64(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One panel of W columns [p0, p0 + W) of the L D L^T elimination (W is a
// compile-time width, so every loop below unrolls without bound checks and
// the LDS loads of a step are issued together).
// (FT threads: the factor kernel's workgroup size)
constexpr int FT = 512;

// n doubles from global memory into LDS, each thread issuing K loads before
// its stores (one memory round trip per K NT entries, not one per NT: these
// one-workgroup kernels run beside bandwidth-heavy ones, where a round trip
// is long)
template <int NT, int K>
__device__ __forceinline__ void copy_to_lds(double* dst, const double* __restrict__ src, int n, int tid) {
    for (int base = 0; base < n; base += NT * K) {
        double v[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int e = base + q * NT + tid;
            v[q] = e < n ? src[e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int e = base + q * NT + tid;
            if (e < n) dst[e] = v[q];
        }
    }
}
template <int W>
__device__ __forceinline__ void chol_panel(double* A, double* dinv, int r, int p0, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    // 1. the diagonal block, one wavefront in registers: lane i < W holds row
    // i of the block (entries j > i are placeholders that are updated but
    // never stored); step k broadcasts the pivot and column k from the lanes
    // that hold them
    if (wave == 0) {
        const int i = min(lane, W - 1);
        double row[W];
#pragma unroll
        for (int j = 0; j < W; ++j) row[j] = A[rm(p0 + i, p0 + min(j, i))];
#pragma unroll
        for (int k = 0; k < W - 1; ++k) {
            const double inv = 1.0 / bcast_f64(row[k], k);
            if (lane == 0) dinv[p0 + k] = inv;
            const double f = row[k] * inv;
#pragma unroll
            for (int j = k + 1; j < W; ++j) row[j] = fma(-f, bcast_f64(row[k], j), row[j]);
        }
        const double last = 1.0 / bcast_f64(row[W - 1], W - 1);
        if (lane == 0) dinv[p0 + W - 1] = last;
        if (lane < W) {
#pragma unroll
            for (int j = 1; j < W; ++j)
                if (j <= lane) A[rm(p0 + lane, p0 + j)] = row[j];
        }
    }
    __syncthreads();
    // 2. the panel's part of every row below the block, a thread per row
    const int pe = p0 + W;
    for (int i = pe + tid; i < r; i += FT) {
        double a[W];
#pragma unroll
        for (int t = 0; t < W; ++t) a[t] = A[rm(i, p0 + t)];
#pragma unroll
        for (int k = 0; k < W - 1; ++k) {
            const double f = a[k] * dinv[p0 + k];
#pragma unroll
            for (int jj = k + 1; jj < W; ++jj) a[jj] = fma(-f, A[rm(p0 + jj, p0 + k)], a[jj]);
        }
#pragma unroll
        for (int t = 0; t < W; ++t) A[rm(i, p0 + t)] = a[t];
    }
    __syncthreads();
    // 3. trailing triangle on the matrix cores: A(i, j) -= sum over the
    // panel's k of (A(i, k) / A(k, k)) A(j, k) for pe <= j <= i, in 16 x 16
    // tiles of the lower part, one wavefront per tile, four k per
    // v_mfma_f64_16x16x4f64 (lane l: row / column l % 16 and k = l / 16 of
    // the operands; rows l / 16 + 4 e of column l % 16 of the result)
    const int nT = (r - pe + 15) >> 4;
    const int lr = lane & 15, lk = lane >> 4;
    for (int t = wave; t < nT * (nT + 1) / 2; t += FT / 64) {
        int I, J;
        tri_rc(t, I, J);
        const int i = pe + 16 * I + lr, j = pe + 16 * J + lr;
        gram_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < W; k0 += 4) {
            const int k = p0 + k0 + lk;
            const double a = i < r ? A[rm(i, k)] * dinv[k] : 0.0;
            const double b = j < r ? A[rm(j, k)] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ii = pe + 16 * I + lk + 4 * e;
            if (ii < r && j <= ii) A[rm(ii, j)] -= acc[e];
        }
    }
    __syncthreads();
}

// L y = g (L unit lower), then q = L^{-T} D^{-1} y for right-hand side c,
// by one wavefront on the factor in LDS (three wavefronts take the three
// coordinates side by side).  NS = row slots in use (64 NS >= r): slot q of a
// lane holds row lane + 64 q; the slot being worked on is a compile-time
// index (the outer loops over it unroll).  The columns go in groups of 16
// (8 for the last ones when r is not a multiple of 16; r is a multiple of
// 8, so no group crosses a slot): a group's LDS entries are requested
// together and their latency is paid once per group, not per column.
template <int NS>
__device__ __forceinline__ void chol_tri(Dev& d, const double* A, const double* dinv, const double* __restrict__ g,
                                         int r, int lane, int c, int zs) {
    double y[NS], di[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = lane + 64 * q;
        di[q] = i < r ? dinv[i] : 0.0;
        y[q] = i < r ? g[i * 3 + c] : 0.0;
    }
    // forward: step k applies column k (y(k) final) to the rows below it;
    // entries outside the strict lower part read the zero at zs (the
    // address is chosen, not the value, so that the loads are unconditional)
#pragma unroll
    for (int qk = 0; qk < NS; ++qk) {
        const int kend = min(r, 64 * qk + 64);
        auto fwd = [&](auto width, int k0) {
            constexpr int GS = decltype(width)::value;
            double cur[GS][NS];
#pragma unroll
            for (int kk = 0; kk < GS; ++kk)
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int i = lane + 64 * q, k = k0 + kk;
                    cur[kk][q] = A[(i > k && i < r) ? rm(i, k) : zs];
                }
#pragma unroll
            for (int kk = 0; kk < GS; ++kk) {
                const int src = (k0 + kk) & 63;
                const double yk = bcast_f64(y[qk] * di[qk], src);
#pragma unroll
                for (int q = qk; q < NS; ++q) y[q] = fma(-cur[kk][q], yk, y[q]);
            }
        };
        int k0 = 64 * qk;
        for (; k0 + 16 <= kend; k0 += 16) fwd(std::integral_constant<int, 16>(), k0);
        if (k0 < kend) fwd(std::integral_constant<int, 8>(), k0);
    }
    // backward: with z = D^{-1} y, q(i) = z(i) - (1 / A(i, i)) sum_{k > i} A(k, i) q(k);
    // acc holds the sums, and row k's value is final when step k broadcasts it
    double acc[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        y[q] *= di[q];
        acc[q] = 0.0;
    }
#pragma unroll
    for (int qk = NS - 1; qk >= 0; --qk) {
        const int ktop = min(r, 64 * qk + 64) - 1;   // r is a multiple of 8
        // columns k0, k0 - 1, ..., k0 - GS + 1
        auto bwd = [&](auto width, int k0) {
            constexpr int GS = decltype(width)::value;
            double cur[GS][NS];
#pragma unroll
            for (int kk = 0; kk < GS; ++kk)
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int i = lane + 64 * q, k = k0 - kk;
                    cur[kk][q] = A[i < k ? rm(k, i) : zs];
                }
#pragma unroll
            for (int kk = 0; kk < GS; ++kk) {
                const int src = (k0 - kk) & 63;
                const double qv = bcast_f64(fma(-di[qk], acc[qk], y[qk]), src);
#pragma unroll
                for (int q = 0; q <= qk; ++q) acc[q] = fma(cur[kk][q], qv, acc[q]);
            }
        };
        int k0 = ktop;
        for (; k0 - 15 >= 64 * qk; k0 -= 16) bwd(std::integral_constant<int, 16>(), k0);
        if (k0 >= 64 * qk) bwd(std::integral_constant<int, 8>(), k0);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = lane + 64 * q;
        if (i < r) {
            const double v = fma(-di[q], acc[q], y[q]);
            d.Qd[i * 3 + c] = v;
            d.Qf[i * 3 + c] = (float)v;
        }
    }
}

// The contact matrix A = Lambda~ + U_C^T diag(W) U_C (packed row-major, from
// k_gram_final) factored in LDS as A = L D L^T without square roots: at
// elimination step k, A(i, j) -= A(i, k) A(j, k) / A(k, k) for k < j <= i,
// so that afterwards L(i, k) = A(i, k) / A(k, k) and D = diag(A).  The
// elimination goes by panels of 16 columns with three barriers each
// (chol_panel); the factor and 1 / D are kept in d.cholf for k_chol_tri.
// Skipped when no collision weight changed since the last factorization
// (wchg clear): the kept factor is still that of A.
__global__ void __launch_bounds__(FT) k_chol_factor(Dev d, const double* __restrict__ Arm,
                                                      const int* __restrict__ n_cv, int* wchg, int* nfact) {
    if (gated(d.gate)) return;
    if (*n_cv == 0 || *wchg == 0) return;
    extern __shared__ double A[];
    const int r = d.r;
    const int tid = threadIdx.x;
    const int tot = r * (r + 1) / 2;
    double* dinv = A + tot;   // 1 / A(k, k) once column k is final
    copy_to_lds<FT, 17>(A, Arm, tot, tid);
    __syncthreads();
    int p0 = 0;
    for (; p0 + CHOL_PANEL <= r; p0 += CHOL_PANEL) chol_panel<CHOL_PANEL>(A, dinv, r, p0, tid);
    if (p0 < r) chol_panel<CHOL_PANEL / 2>(A, dinv, r, p0, tid);   // r is a multiple of 8
    for (int e = tid; e < tot + r; e += FT) d.cholf[e] = A[e];
    if (tid == 0) {
        *wchg = 0;   // every thread read the flag before the first barrier above
        atomicAdd(nfact, 1);
    }
}

// q = A^{-1} g for the three coordinates (Eq. (subspace_collision)), in one
// workgroup: three wavefronts solve on the kept factor (chol_tri), loaded
// into LDS.  Without contact vertices A = Lambda~, whose precomputed inverse
// is applied instead.
// NS: row slots of the solve, 2 for r <= 128 and 3 up to MAX_R (chosen on
// the host; one instantiation per kernel keeps it within 128 VGPRs).
template <int NS>
__global__ void __launch_bounds__(1024) k_chol_tri(Dev d, const int* __restrict__ n_cv) {
    if (gated(d.gate)) return;
    extern __shared__ double A[];
    const int r = d.r;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tot = r * (r + 1) / 2;
    // g = U^T r0 (summed into d.gvec before the factor was waited for),
    // kept in LDS after the factor
    double* g = A + tot + r + 1;
    for (int o = tid; o < 3 * r; o += 1024) g[o] = d.gvec[o];
    if (*n_cv == 0) {
        __syncthreads();   // g complete
        // q = A^{-1} g: wavefront w takes rows w, w + 16, ..., lanes the
        // columns lane + 64 s; g is loaded once and the rows four at a time
        // (addresses clamped into the matrix, the extra entries multiplied
        // by 0), each row then reduced across the wavefront
        constexpr int RW = 4 * NS;   // rows per wavefront: 16 RW >= 64 NS >= r
        double gj[NS][3];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int j = lane + 64 * q, jc = min(j, r - 1);
            const double m = j < r ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) gj[q][c] = g[jc * 3 + c] * m;
        }
#pragma unroll
        for (int t0 = 0; t0 < RW; t0 += 4) {
            double a[4][NS];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int q = 0; q < NS; ++q)
                    a[t][q] = d.Ainv[(size_t)min(wave + 16 * (t0 + t), r - 1) * r + min(lane + 64 * q, r - 1)];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = wave + 16 * (t0 + t);
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    s0 = fma(a[t][q], gj[q][0], s0);
                    s1 = fma(a[t][q], gj[q][1], s1);
                    s2 = fma(a[t][q], gj[q][2], s2);
                }
                for (int o = 32; o > 0; o >>= 1) {
                    s0 += __shfl_xor(s0, o);
                    s1 += __shfl_xor(s1, o);
                    s2 += __shfl_xor(s2, o);
                }
                if (lane == 0 && row < r) {
                    d.Qd[row * 3] = s0;
                    d.Qd[row * 3 + 1] = s1;
                    d.Qd[row * 3 + 2] = s2;
                    d.Qf[row * 3] = (float)s0;
                    d.Qf[row * 3 + 1] = (float)s1;
                    d.Qf[row * 3 + 2] = (float)s2;
                }
            }
        }
        return;
    }
    double* dinv = A + tot;
    const int zs = tot + r;   // a zero entry for the solves
    copy_to_lds<1024, 9>(A, d.cholf, tot + r, tid);
    if (tid == 0) A[zs] = 0.0;
    __syncthreads();
    if (wave >= 3) return;   // wavefront c solves for coordinate c
    chol_tri<NS>(d, A, dinv, g, r, lane, wave, zs);
}


__global__ void k_aos4(int n, const float* __restrict__ X, float4* X4) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        X4[v] = make_float4(X[v], X[n + v], X[2 * n + v], 0.f);
}

__global__ void k_copy_i32(const int* __restrict__ gate, int* __restrict__ dst, const int* __restrict__ src, int n) {
    if (gated(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// previous constraint set <- current (count from device)
__global__ void k_save_prev(const int* __restrict__ gate, int* cnt, const int2* __restrict__ cp, const int* __restrict__ a, int2* pp, int* pa,
                            int first) {
    if (gated(gate)) return;
    const int nc = first ? 0 : cnt[2] + cnt[3];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
        pp[i] = cp[i];
        pa[i] = a[i];
    }
}

// bookkeeping of the device counters at the start of an outer stage
__global__ void k_stage_counters(const int* __restrict__ gate, int* cnt, int first, unsigned long long* tmin_bits) {
    if (gated(gate)) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt[4] = first ? 0 : cnt[2];
        cnt[5] = first ? 0 : cnt[3];
        cnt[0] = 0;
        cnt[1] = 0;
        cnt[10] = 0;
        if (first) tmin_bits[1] = (unsigned long long)__double_as_longlong(NOHIT);
        tmin_bits[0] = (unsigned long long)__double_as_longlong(NOHIT);
    }
}

__global__ void k_sum2(const int* __restrict__ gate, int* cnt) {
    if (gated(gate)) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) cnt[9] = cnt[0] + cnt[1];
}

// ================================================================ tangle check
// Debug check of an end state: an edge that crosses a triangle sharing none
// of its vertices means two triangles intersect.  Orientation signs in FP64
// (the FP32 coordinates and their differences are exact there) with a
// static error bound; a sign the bound cannot certify makes the pair
// "undecided", which is counted apart and never reported as a tangle.
__device__ __forceinline__ int orient_sign(double4 a, double4 b, double4 c, double4 p) {
    const double bx = b.x - a.x, by = b.y - a.y, bz = b.z - a.z;
    const double cx = c.x - a.x, cy = c.y - a.y, cz = c.z - a.z;
    const double px = p.x - a.x, py = p.y - a.y, pz = p.z - a.z;
    const double m0 = cy * pz - cz * py, m1 = cx * pz - cz * px, m2 = cx * py - cy * px;
    const double det = bx * m0 - by * m1 + bz * m2;
    const double perm = fabs(bx) * (fabs(cy * pz) + fabs(cz * py)) + fabs(by) * (fabs(cx * pz) + fabs(cz * px)) +
                        fabs(bz) * (fabs(cx * py) + fabs(cy * px));
    const double bound = 1e-14 * perm;
    return det > bound ? 1 : (det < -bound ? -1 : 0);
}

__device__ __forceinline__ double4 to_d4(float4 v) { return make_double4(v.x, v.y, v.z, 0.0); }

// closed segment pq against closed triangle abc: 1 crossing, 0 apart, -1 undecided
__device__ __forceinline__ int segment_crosses_triangle(double4 p, double4 q, double4 a, double4 b, double4 c) {
    const int sp = orient_sign(a, b, c, p), sq = orient_sign(a, b, c, q);
    if (sp == 0 || sq == 0) return -1;
    if (sp == sq) return 0;
    const int o1 = orient_sign(p, q, a, b), o2 = orient_sign(p, q, b, c), o3 = orient_sign(p, q, c, a);
    if (o1 == 0 || o2 == 0 || o3 == 0) return -1;
    return (o1 == o2 && o2 == o3) ? 1 : 0;
}

// One group of G lanes per edge, triangles from the cell buckets (static
// boxes of the state, the triangle grid).  cnt[CNT_TANGLES]: crossings,
// cnt[CNT_TANGLES + 1]: undecided pairs and queries beyond their work bound;
// a crossing flags the running step.
template <int G>
__global__ void __launch_bounds__(256) k_tangle_query(Dev d, const float* __restrict__ ebox,
                                                      const BpGrid* __restrict__ gp, const int* __restrict__ bptr,
                                                      const BpRec* __restrict__ rec, int P,
                                                      const float4* __restrict__ x4, int* cnt) {
    constexpr int GPB = 256 / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int sub = (threadIdx.x & 63) / G;
    const int q = xcd_block(blockIdx.x, gridDim.x) * GPB + grp;
    const BpGrid g = *gp;
    int crossings = 0, undecided = 0;
    if (q < d.ne) {
        const double4 p0 = to_d4(x4[d.edges[2 * q]]), p1 = to_d4(x4[d.edges[2 * q + 1]]);
        bool full = false;
        group_query<false, G, true>(d, q, lane, sub, ebox, g, bptr, rec, P, MAX_VISIT, full, [&](int, int id) {
            const TriRec tr = d.tri[id];
            const int r = segment_crosses_triangle(p0, p1, to_d4(x4[tr.v0]), to_d4(x4[tr.v1]), to_d4(x4[tr.v2]));
            crossings += r > 0;
            undecided += r < 0;
        });
        if (full && lane == 0) undecided += 1;
    }
    if (crossings) {
        atomicAdd(&cnt[CNT_TANGLES], crossings);
        atomicOr(&cnt[CNT_STEP_FAIL], STEP_TANGLED);
    }
    if (undecided) atomicAdd(&cnt[CNT_TANGLES + 1], undecided);
}

// ================================================================ host side

// lanes per query of the counting pass, and its grid (one group per query)
constexpr int QUERY_LANES = 8;   // lanes per query of the tangle check (the broad phase's are c.qlanes)
static inline int qblocks(int64_t nq, int G = QUERY_LANES) {
    return (int)std::max<int64_t>(1, (nq + 256 / G - 1) / (256 / G));
}



static inline int gblocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, GRID_LOOP));
}

// the heavy queries are few: one workgroup per CU takes them (each
// workgroup also counts itself out once, for the list's reset)
static inline int rescan_blocks(int64_t nq) { return std::min(gblocks(nq), 256); }
// grids of the grid-stride kernels over the constraint set (at most a few
// per vertex in practice; sized for one pass at one constraint per vertex)
// and over the candidate lists (one pass at four per vertex): capacity-sized
// grids would launch thousands of idle workgroups on small scenes
static inline int cgrid(const Scene& s, const ContactState& c) {
    return std::min(gblocks(c.ccap), gblocks(s.nv));
}
static inline int candgrid(const Scene& s, const ContactState& c) {
    return std::min(gblocks(2 * c.cap), gblocks(4 * (int64_t)s.nv));
}

#define HC(expr)                                                                                        \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return set_error(CLOTH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

bool contact_enabled(const Scene& s, const ContactState& c) { return c.nob > 0 || s.self_contact; }

cloth_status contact_layout(Scene& s, ContactState& c, const Carver& carve) {
    const int n = s.nv;
    c.cap = s.pair_cap;
    int P = 1;
    while (P < 2 * std::max(s.nt, s.ne)) P <<= 1;
    c.hash_p = P;
    // per-query output bound: the int prefix sums over queries cannot overflow
    c.max_out = (int)std::min<int64_t>(1024, (int64_t)0x7fffffff / std::max<int64_t>(1, std::max(n, s.ne)) - 1);
    // (the largest scan: the keep flags over both candidate lists, or with
    // the reusable superset over both superset lists)
    const int64_t kmul = s.bp_reuse ? 4 : 2;
    int64_t maxscan = std::max<int64_t>({kmul * c.cap, (int64_t)n + 1, (int64_t)s.ne + 1, (int64_t)P + 1});
    c.ntiles_cap = (int)((maxscan + SCAN_TILE - 1) / SCAN_TILE) + 1;
    auto I = [&](size_t k) { return static_cast<int*>(carve(sizeof(int) * k)); };
    const int rw = std::max(s.r, s.r_warm);   // the warm-start basis may be wider
    c.gpart2 = static_cast<double*>(carve(sizeof(double) * ((size_t)(s.nblk + 31) / 32 + 1) * rw * 3));
    c.gvec = static_cast<double*>(carve(sizeof(double) * rw * 3));
    c.cnt = I(CNT_WORDS);
    c.tmin_bits = static_cast<unsigned long long*>(carve(32));
    c.tpart = static_cast<double*>(carve(sizeof(double) * 2 * GRID_LOOP));
    c.s_dev = static_cast<double*>(carve(8));
    c.scan_tiles = I(c.ntiles_cap);
    c.ob_a = I((size_t)MAX_OBST * n);
    c.ob_dev = static_cast<ObstD*>(carve(sizeof(ObstD) * MAX_OBST));
    if (!c.gpart2 || !c.gvec || !c.cnt || !c.tmin_bits || !c.tpart || !c.s_dev || !c.scan_tiles || !c.ob_a || !c.ob_dev)
        return set_error(CLOTH_E_OOM, "arena exhausted (contact scalars)");
    Dev& d = s.d;
    d.gvec = c.gvec;
    d.fail = c.cnt + CNT_STEP_FAIL;
    d.ob_a = c.ob_a;
    d.ob = c.ob_dev;
    d.nob = 0;
    d.kc = (float)s.kc;
    d.Kb = (float)s.Kb;
    d.dhat = s.dhat;
    c.enabled = contact_enabled(s, c);
    // pair buffers only when self contact is on; obstacles need only per-vertex data
    int64_t pc = s.self_contact ? c.cap : 1;
    c.cap = pc;
    // constraints (kept candidates, VT + EE) are a small fraction of the
    // candidates (under one per vertex in the drapes, against ten or more
    // candidates): their lists get an eighth of the candidate capacity
    const int64_t cc = s.self_contact ? std::max<int64_t>(4096, pc / 8) : 1;
    c.ccap = cc;
    c.vbox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(s.self_contact ? n : 1)));
    c.tbox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(s.self_contact ? s.nt : 1)));
    c.ebox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(s.self_contact ? s.ne : 1)));
    const size_t mt = s.self_contact ? (size_t)std::max(s.nt, s.ne) : 1;
    c.bucket_cnt = I((size_t)P + 1);
    c.bucket_ptr = I((size_t)P + 1);
    c.rec = static_cast<BpRec*>(carve(sizeof(BpRec) * mt));
    c.qscratch = I((size_t)QK * (s.self_contact ? (size_t)std::max(n, s.ne) : 1));
    c.heavy_q = I(s.self_contact ? (size_t)std::max(n, s.ne) : 1);
    c.bpart = static_cast<float*>(carve(sizeof(float) * BP_PART * GRID_LOOP));
    c.xm4 = static_cast<float4*>(carve(sizeof(float4) * (s.self_contact ? (size_t)n : 1)));
    c.xp4 = static_cast<float4*>(carve(sizeof(float4) * (s.self_contact ? (size_t)n : 1)));
    c.grid = static_cast<BpGrid*>(carve(sizeof(BpGrid) * 2));
    c.vcount = I((size_t)n + 1);
    c.ecount = I((size_t)s.ne + 1);
    c.cand_vt = static_cast<int2*>(carve(sizeof(int2) * pc));
    c.cand_ee = static_cast<int2*>(carve(sizeof(int2) * pc));
    // the reusable superset (only when used): grown boxes and lists of twice
    // the candidate capacity
    const bool sup = s.self_contact && s.bp_reuse;
    c.svbox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(sup ? n : 1)));
    c.stbox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(sup ? s.nt : 1)));
    c.sebox = static_cast<float*>(carve(sizeof(float) * 6 * (size_t)(sup ? s.ne : 1)));
    c.sup_vt = static_cast<int2*>(carve(sizeof(int2) * (sup ? 2 * pc : 1)));
    c.sup_ee = static_cast<int2*>(carve(sizeof(int2) * (sup ? 2 * pc : 1)));
    c.supw = I(16);
    c.toi_sched = I(8 * TOI_LINE);
    c.sup_mu0 = s.bp_mu0;
    c.sup_kappa = s.bp_kappa;
    c.sup_on = s.bp_reuse != 0;
    c.toi_vt = static_cast<double*>(carve(sizeof(double) * pc));
    c.toi_ee = static_cast<double*>(carve(sizeof(double) * pc));
    c.keep = I(std::max<int64_t>((sup ? 4 : 2) * pc, (int64_t)std::max(n, s.ne) + 1));
    c.keep_ofs = I((sup ? 4 : 2) * pc);
    c.cand_a = I(2 * pc);
    c.cpair = static_cast<int2*>(carve(sizeof(int2) * cc));
    c.cpair_prev = static_cast<int2*>(carve(sizeof(int2) * cc));
    c.ca = I(cc);
    c.ca_prev = I(cc);
    c.clam = static_cast<double2*>(carve(sizeof(double2) * cc));
    c.cnrm = static_cast<float4*>(carve(sizeof(float4) * cc));
    c.slot = static_cast<float4*>(carve(sizeof(float4) * 4 * cc));
    c.vslot_ptr = I((size_t)n + 1);
    c.vslot_fill = I((size_t)n + 1);
    c.vslot = I(4 * cc);
    c.cvlist = I((size_t)n + 1);
    c.cvflag = I((size_t)n + 1);
    c.cvofs = I((size_t)n + 1);
    if (!c.vbox || !c.tbox || !c.ebox || !c.bucket_cnt || !c.bucket_ptr || !c.rec || !c.qscratch || !c.heavy_q ||
        !c.bpart || !c.grid || !c.xm4 || !c.xp4 || !c.vcount || !c.ecount || !c.cand_vt || !c.cand_ee || !c.toi_vt ||
        !c.toi_ee || !c.keep || !c.keep_ofs || !c.cand_a || !c.cpair || !c.cpair_prev || !c.ca ||
        !c.ca_prev || !c.clam || !c.cnrm || !c.slot || !c.vslot_ptr || !c.vslot_fill || !c.vslot || !c.cvlist ||
        !c.cvflag || !c.cvofs || !c.svbox || !c.stbox || !c.sebox || !c.sup_vt || !c.sup_ee || !c.supw ||
        !c.toi_sched)
        return set_error(CLOTH_E_OOM, "arena exhausted (contact buffers)");
    d.vslot_ptr = c.vslot_ptr;
    d.vslot = c.vslot;
    d.slot = c.slot;
    // chunks of at least GRAM_MIN_PER_CHUNK contact vertices: no more than
    // the vertices can fill
    c.gram_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(GRAM_CHUNKS, (s.nv + GRAM_MIN_PER_CHUNK - 1) /
                                                                              GRAM_MIN_PER_CHUNK));
    return CLOTH_OK;
}

cloth_status contact_upload(Scene& s, ContactState& c) {
    const int n = s.nv;
    HC(hipMemset(c.cnt, 0, sizeof(int) * CNT_WORDS));
    // no superset yet: the first stage builds it
    const int supw0[16] = {0, 0, 1};
    HC(hipMemcpy(c.supw, supw0, sizeof(supw0), hipMemcpyHostToDevice));
    HC(hipMemset(c.ob_a, 0xff, sizeof(int) * (size_t)MAX_OBST * n));
    std::vector<unsigned long long> tb(4, 0x4000000000000000ull);  // 2.0
    HC(hipMemcpy(c.tmin_bits, tb.data(), 32, hipMemcpyHostToDevice));
    double one = 1.0;
    HC(hipMemcpy(c.s_dev, &one, 8, hipMemcpyHostToDevice));
    HC(hipMemset(c.vslot_ptr, 0, sizeof(int) * (n + 1)));
    HC(hipFuncSetAttribute((const void*)k_chol_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)chol_lds_bytes(s.r)));
    HC(hipFuncSetAttribute((const void*)k_chol_tri<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)(chol_lds_bytes(s.r) + sizeof(double) * 3 * s.r)));
    HC(hipFuncSetAttribute((const void*)k_chol_tri<3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)(chol_lds_bytes(s.r) + sizeof(double) * 3 * s.r)));
    return CLOTH_OK;
}

cloth_status contact_set_obstacles(Scene& s, ContactState& c) {
    c.nob = (int)s.obst.size();
    for (int j = 0; j < c.nob; ++j) c.ob[j] = s.obst[j];
    HC(hipMemcpy(c.ob_dev, c.ob, sizeof(ObstD) * MAX_OBST, hipMemcpyHostToDevice));
    s.d.nob = c.nob;
    c.enabled = contact_enabled(s, c);
    return CLOTH_OK;
}

// Boxes of the vertices, triangles and edges over (xm, xp) grown by dhat,
// and the cell sizes of the two target families (the tangle check's boxes:
// no reusable-list check).
static void bp_boxes(Scene& s, ContactState& c, const float* xm, const float* xp, float dhat, hipStream_t st) {
    Dev& d = s.d;
    const int n = s.nv;
    const int nbb = gblocks((int64_t)n + s.nt + s.ne);
    // AoS copies of the two positions, for the corner gathers of the boxes and the TOI
    hipLaunchKernelGGL(k_aos_pair, dim3(gblocks(n)), dim3(TPB), 0, st, s.d.gate, n, xm, xp, c.xm4, c.xp4);
    hipLaunchKernelGGL(k_boxes, dim3(nbb), dim3(256), 0, st, d, (const float4*)c.xm4, (const float4*)c.xp4,
                       dhat, c.vbox, c.tbox, c.ebox, c.bpart, (const float*)nullptr, (const float*)nullptr,
                       (const float*)nullptr, (int*)nullptr);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(256), 0, st, s.d.gate, (const float*)c.bpart, nbb, s.nt, s.ne, c.grid);
}

// Files the targets of one family (vt: triangles, else edges; boxes tb) in
// the cell buckets: counts, bucket offsets, inline records.
static cloth_status bp_file_targets(Scene& s, ContactState& c, bool vt, const float* tb, hipStream_t st) {
    Dev& d = s.d;
    const int P = c.hash_p;
    const int m = vt ? s.nt : s.ne;
    const BpGrid* g = c.grid + (vt ? 0 : 1);
    hipLaunchKernelGGL(k_fill_i32, dim3(gblocks(P + 1)), dim3(TPB), 0, st, s.d.gate, c.bucket_cnt, 0, P + 1);
    hipLaunchKernelGGL(k_cells, dim3(gblocks(m)), dim3(TPB), 0, st, s.d.gate, m, tb, g, c.bucket_cnt, P, c.cnt + 7);
    HC(scan_exclusive(c.bucket_cnt, c.bucket_ptr, P + 1, nullptr, c.scan_tiles, nullptr, s.d.gate, st));
    hipLaunchKernelGGL(k_copy_i32, dim3(gblocks(P + 1)), dim3(TPB), 0, st, s.d.gate, c.bucket_cnt, c.bucket_ptr, P + 1);
    hipLaunchKernelGGL(k_bucket_fill, dim3(gblocks(m)), dim3(TPB), 0, st, d, vt ? 1 : 0, m, tb, g, P,
                       c.bucket_cnt, c.rec);
    return CLOTH_OK;
}

// the counting and writing passes with G lanes per query (4, 8 or 16, a
// scene setting the autotuner picks; the candidate lists do not depend on it)
template <int G>
static void query_passes(Scene& s, ContactState& c, bool vt, const float* qb, const BpGrid* g, int* cnts, int2* outp,
                         int* n_out, int64_t cap, bool timed_ee, hipStream_t st) {
    Dev& d = s.d;
    const int nq = vt ? s.nv : s.ne;
    const int P = c.hash_p;
    if (vt)
        hipLaunchKernelGGL((k_query_count<true, G>), dim3(qblocks(nq, G)), dim3(256), 0, st, d, qb, g, c.bucket_ptr,
                           c.rec, P, cnts, c.qscratch, c.max_out, c.cnt + 7, c.heavy_q, c.cnt + HEAVY_SLOT);
    else {
        if (timed_ee) {
            timing_end(s, st);
            timing_begin(s, K_QUERY_EE, st);
        }
        launch_timed(k_query_count<false, G>, dim3(qblocks(nq, G)), dim3(256), 0, st, d, qb, g,
                     (const int*)c.bucket_ptr, (const BpRec*)c.rec, P, cnts, c.qscratch, c.max_out, c.cnt + 7,
                     c.heavy_q, c.cnt + HEAVY_SLOT);
        if (timed_ee) {
            timing_end(s, st);
            timing_begin(s, K_BROAD, st);
        }
    }
    hipLaunchKernelGGL(k_copy_i32, dim3(gblocks(nq)), dim3(TPB), 0, st, s.d.gate, c.keep, cnts, nq);
    (void)scan_exclusive(c.keep, cnts, nq, nullptr, c.scan_tiles, nullptr, s.d.gate, st);
    hipLaunchKernelGGL(k_count_total, dim3(1), dim3(64), 0, st, s.d.gate, cnts, c.keep, nq, n_out + (vt ? 0 : 1), cap,
                       c.cnt + 7);
    hipLaunchKernelGGL(k_query_copy<G>, dim3(qblocks(nq, G)), dim3(256), 0, st, s.d.gate, nq, (const int*)cnts,
                       (const int*)c.keep, (const int*)c.qscratch, outp, cap);
}

// Sorted VT and EE pairs of the boxes (vb: vertices, tb: triangles, eb:
// edges) that overlap, into out_vt / out_ee with their counts in n_out[0],
// n_out[1]; per-query offsets in c.vcount / c.ecount.  The grid comes from
// the box statistics in c.bpart.  Gated by s.d.gate.
static cloth_status bp_pairs(Scene& s, ContactState& c, const float* vb, const float* tb, const float* eb,
                             int2* out_vt, int2* out_ee, int* n_out, int64_t cap, hipStream_t st) {
    Dev& d = s.d;
    const int n = s.nv;
    const int P = c.hash_p;
    const int nbb = gblocks((int64_t)n + s.nt + s.ne);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(256), 0, st, s.d.gate, (const float*)c.bpart, nbb, s.nt, s.ne, c.grid);
    for (int pass = 0; pass < 2; ++pass) {
        const bool vt = pass == 0;
        const BpGrid* g = c.grid + (vt ? 0 : 1);
        cloth_status rc = bp_file_targets(s, c, vt, vt ? tb : eb, st);
        if (rc != CLOTH_OK) return rc;
        const int nq = vt ? n : s.ne;
        int* cnts = vt ? c.vcount : c.ecount;
        int2* outp = vt ? out_vt : out_ee;
        const float* qb = vt ? vb : eb;
        if (c.qlanes == 4)
            query_passes<4>(s, c, vt, qb, g, cnts, outp, n_out, cap, true, st);
        else if (c.qlanes == 16)
            query_passes<16>(s, c, vt, qb, g, cnts, outp, n_out, cap, true, st);
        else
            query_passes<8>(s, c, vt, qb, g, cnts, outp, n_out, cap, true, st);
        if (vt)
            hipLaunchKernelGGL(k_query_rescan<true>, dim3(rescan_blocks(nq)), dim3(TPB), 0, st, d, qb, g, c.bucket_ptr,
                               c.rec, P, (const int*)cnts, (const int*)c.keep, outp, cap, c.max_out, c.cnt + 7,
                               (const int*)c.heavy_q, c.cnt + HEAVY_SLOT);
        else
            hipLaunchKernelGGL(k_query_rescan<false>, dim3(rescan_blocks(nq)), dim3(TPB), 0, st, d, qb, g, c.bucket_ptr,
                               c.rec, P, (const int*)cnts, (const int*)c.keep, outp, cap, c.max_out, c.cnt + 7,
                               (const int*)c.heavy_q, c.cnt + HEAVY_SLOT);
    }
    HC(hipGetLastError());
    return CLOTH_OK;
}

// Broad phase on (xm, xp) -> sorted candidates, counts in cnt[0], cnt[1],
// per-query offsets in c.vcount / c.ecount: stage boxes (checked against the
// reusable superset's boxes), a rebuild of the superset on grown boxes when
// a box escaped (launched always, gated on the device), then the superset
// filtered by the stage boxes.
static cloth_status broad_phase(Scene& s, ContactState& c, const float* xm, const float* xp, hipStream_t st) {
    if (!s.self_contact) return CLOTH_OK;
    Dev& d = s.d;
    const int n = s.nv;
    const int nbb = gblocks((int64_t)n + s.nt + s.ne);
    if (!c.sup_on) {
        // pairs of the stage boxes themselves
        hipLaunchKernelGGL(k_aos_pair, dim3(gblocks(n)), dim3(TPB), 0, st, s.d.gate, n, xm, xp, c.xm4, c.xp4);
        hipLaunchKernelGGL(k_boxes, dim3(nbb), dim3(256), 0, st, d, (const float4*)c.xm4, (const float4*)c.xp4,
                           (float)s.dhat, c.vbox, c.tbox, c.ebox, c.bpart, (const float*)nullptr,
                           (const float*)nullptr, (const float*)nullptr, (int*)nullptr);
        return bp_pairs(s, c, c.vbox, c.tbox, c.ebox, c.cand_vt, c.cand_ee, c.cnt, c.cap, st);
    }
    hipLaunchKernelGGL(k_aos_pair, dim3(gblocks(n)), dim3(TPB), 0, st, s.d.gate, n, xm, xp, c.xm4, c.xp4);
    hipLaunchKernelGGL(k_boxes, dim3(nbb), dim3(256), 0, st, d, (const float4*)c.xm4, (const float4*)c.xp4,
                       (float)s.dhat, c.vbox, c.tbox, c.ebox, c.bpart, (const float*)c.svbox, (const float*)c.stbox,
                       (const float*)c.sebox, c.supw + 2);
    hipLaunchKernelGGL(k_sup_gate, dim3(1), dim3(64), 0, st, (const int*)s.d.gate, c.supw, (const int*)c.cnt);
    const int* const stage_gate = s.d.gate;
    for (int attempt = 0; attempt < 2; ++attempt) {
        // the rebuild (gated by supw[5]), then its retry without margins
        // (gated by supw[9])
        if (attempt == 1) hipLaunchKernelGGL(k_sup_retry, dim3(1), dim3(64), 0, st, c.supw, c.cnt);
        s.d.gate = c.supw + (attempt == 0 ? 5 : 9);
        hipLaunchKernelGGL(k_sup_grow, dim3(nbb), dim3(256), 0, st, s.d, (const float4*)c.xm4, (const float4*)c.xp4,
                           (const float*)c.vbox, (const float*)c.tbox, (const float*)c.ebox, c.svbox, c.stbox,
                           c.sebox, c.bpart, (float)c.sup_mu0, (float)c.sup_kappa, (const int*)(c.supw + 7));
        cloth_status rc = bp_pairs(s, c, c.svbox, c.stbox, c.sebox, c.sup_vt, c.sup_ee, c.supw, 2 * c.cap, st);
        hipLaunchKernelGGL(k_sup_done, dim3(1), dim3(64), 0, st, (const int*)s.d.gate, c.supw, (const int*)c.cnt);
        s.d.gate = stage_gate;
        if (rc != CLOTH_OK) return rc;
    }
    const int64_t scap = 4 * c.cap;   // both superset lists
    const int fb = gblocks(scap);
    hipLaunchKernelGGL(k_sup_filter, dim3(fb), dim3(256), 0, st, c.supw, (const int2*)c.sup_vt, (const int2*)c.sup_ee,
                       (const float*)c.vbox, (const float*)c.tbox, (const float*)c.ebox, n, s.nt, s.ne, c.keep);
    HC(scan_exclusive(c.keep, c.keep_ofs, (int)scap, c.supw + 4, c.scan_tiles, nullptr, c.supw + 6, st));
    hipLaunchKernelGGL(k_sup_compact, dim3(fb), dim3(256), 0, st, (const int*)c.supw, (const int2*)c.sup_vt,
                       (const int2*)c.sup_ee, (const int*)c.keep, (const int*)c.keep_ofs, c.cand_vt, c.cand_ee, c.cnt,
                       c.cap);
    hipLaunchKernelGGL(k_query_ofs, dim3(gblocks((int64_t)n + s.ne)), dim3(256), 0, st, (const int*)c.supw,
                       (const int*)c.cnt, (const int2*)c.cand_vt, (const int2*)c.cand_ee, n, s.ne, c.vcount, c.ecount);
    HC(hipGetLastError());
    return CLOTH_OK;
}

// Debug tangle check of the positions x (end of a step): static boxes,
// triangles filed in their grid, one query per edge (k_tangle_query).
// The broad-phase buffers are free at this point of the step.
cloth_status contact_tangle_check(Scene& s, ContactState& c, const float* x, hipStream_t st) {
    if (!s.self_contact) return CLOTH_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, (const int*)nullptr, c.cnt + CNT_TANGLES, 0, 2);
    bp_boxes(s, c, x, x, 0.0f, st);
    cloth_status rc = bp_file_targets(s, c, true, c.tbox, st);
    if (rc != CLOTH_OK) return rc;
    hipLaunchKernelGGL(k_tangle_query<QUERY_LANES>, dim3(qblocks(s.ne)), dim3(256), 0, st, s.d,
                       (const float*)c.ebox, (const BpGrid*)c.grid, (const int*)c.bucket_ptr, (const BpRec*)c.rec,
                       c.hash_p, (const float4*)c.xm4, c.cnt);
    HC(hipGetLastError());
    return CLOTH_OK;
}

// TOI + merge with the previous set + obstacles + step length + compaction +
// filter x = xm + s (xp - xm) written to d.x and d.xm.
static cloth_status toi_merge_filter(Scene& s, ContactState& c, const float* xm, const float* xp,
                                    unsigned long long* dxo, hipStream_t st) {
    Dev& d = s.d;
    const int n = s.nv;
    int npart = 0;
    if (s.self_contact) {
        const int nb = gblocks(2 * c.cap);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, s.d.gate, c.toi_sched, 0, 8 * TOI_LINE);
        timing_begin(s, K_TOI, st);
        launch_timed(k_toi_merge, dim3(nb), dim3(TPB), 0, st, d, (const float4*)c.xm4, (const float4*)c.xp4,
                     (const int2*)c.cand_vt, (const int2*)c.cand_ee, c.cnt, c.toi_vt, c.toi_ee, c.keep,
                     c.cand_a, c.tpart, 1, c.toi_sched);
        timing_end(s, st);
        timing_begin(s, K_OUTER, st);
        hipLaunchKernelGGL(k_prev_match, dim3(gblocks(c.ccap)), dim3(TPB), 0, st, s.d.gate, (const int*)c.cnt,
                           (const int2*)c.cpair_prev, (const int*)c.ca_prev, (const int2*)c.cand_vt,
                           (const int2*)c.cand_ee, (const int*)c.vcount, (const int*)c.ecount, n, s.ne, c.keep,
                           c.cand_a);
        npart = nb;
    }
    else
        timing_begin(s, K_OUTER, st);
    if (c.nob > 0) {
        const int nb = gblocks(n);
        hipLaunchKernelGGL(k_obstacles_outer, dim3(nb), dim3(TPB), 0, st, d, xm, xp, c.tpart + npart, c.cnt + 10);
        npart += nb;
    }
    hipLaunchKernelGGL(k_step_length, dim3(1), dim3(256), 0, st, s.d.gate, (const double*)c.tpart, npart, c.tmin_bits, s.alpha,
                       c.s_dev, (const int*)(c.cnt + CNT_STEP_FAIL));
    if (s.self_contact) {
        hipLaunchKernelGGL(k_sum2, dim3(1), dim3(64), 0, st, s.d.gate, c.cnt);
        HC(scan_exclusive(c.keep, c.keep_ofs, (int)(2 * c.cap), c.cnt + 9, c.scan_tiles, nullptr, s.d.gate, st));
        hipLaunchKernelGGL(k_compact, dim3(candgrid(s, c)), dim3(TPB), 0, st, s.d.gate, c.cand_vt, c.cand_ee, c.cnt, c.keep,
                           c.keep_ofs, c.cand_a, c.cpair, c.ca, c.ccap);
    }
    HC(launch_filter(d, xm, xp, c.s_dev, d.x, d.xm, dxo, st));
    HC(hipGetLastError());
    return CLOTH_OK;
}

// Per block: frozen data at x-, vertex slot lists, contact-vertex list.
static cloth_status block_setup(Scene& s, ContactState& c, hipStream_t st) {
    Dev& d = s.d;
    const int n = s.nv;
    if (s.self_contact) {
        hipLaunchKernelGGL(k_freeze, dim3(cgrid(s, c)), dim3(TPB), 0, st, d, c.cnt, c.cpair, c.clam, c.cnrm);
        hipLaunchKernelGGL(k_fill_i32, dim3(gblocks(n + 1)), dim3(TPB), 0, st, s.d.gate, c.vslot_fill, 0, n + 1);
        hipLaunchKernelGGL(k_slot_count, dim3(cgrid(s, c)), dim3(TPB), 0, st, d, c.cnt, c.cpair, c.vslot_fill);
        HC(scan_exclusive(c.vslot_fill, c.vslot_ptr, n + 1, nullptr, c.scan_tiles, nullptr, s.d.gate, st));
        hipLaunchKernelGGL(k_copy_i32, dim3(gblocks(n + 1)), dim3(TPB), 0, st, s.d.gate, c.vslot_fill, c.vslot_ptr, n + 1);
        hipLaunchKernelGGL(k_slot_fill, dim3(cgrid(s, c)), dim3(TPB), 0, st, d, c.cnt, c.cpair, c.vslot_fill,
                           c.vslot);
    }
    hipLaunchKernelGGL(k_slot_sort, dim3(gblocks(n)), dim3(TPB), 0, st, d, c.vslot_ptr, c.vslot, c.ob_a, c.nob,
                       c.cvflag);
    HC(scan_exclusive(c.cvflag, c.cvofs, n, nullptr, c.scan_tiles, nullptr, s.d.gate, st));
    hipLaunchKernelGGL(k_cv_compact, dim3(gblocks(n)), dim3(TPB), 0, st, s.d.gate, n, c.cvflag, c.cvofs, c.cvlist, c.cnt + 6,
                       c.cnt + CNT_WCHG);
    HC(hipGetLastError());
    c.active = true;
    return CLOTH_OK;
}

// Timing brackets of a stage: K_BROAD from the start to the end of the
// broad phase (closed and reopened around the edge-edge counting pass,
// K_QUERY_EE), K_TOI around the TOI kernel, K_OUTER from there to the end.
static cloth_status outer_stage(Scene& s, ContactState& c, const float* xm, const float* xp, bool first,
                                bool setup, unsigned long long* dxo, hipStream_t st) {
    timing_begin(s, K_BROAD, st);
    if (first) hipLaunchKernelGGL(k_fill_i32, dim3(gblocks((int64_t)MAX_OBST * s.nv)), dim3(TPB), 0, st, s.d.gate, c.ob_a, -1,
                                  MAX_OBST * s.nv);
    hipLaunchKernelGGL(k_save_prev, dim3(cgrid(s, c)), dim3(TPB), 0, st, s.d.gate, c.cnt, c.cpair, c.ca, c.cpair_prev,
                       c.ca_prev, first ? 1 : 0);
    hipLaunchKernelGGL(k_stage_counters, dim3(1), dim3(64), 0, st, s.d.gate, c.cnt, first ? 1 : 0, c.tmin_bits);
    cloth_status rc = broad_phase(s, c, xm, xp, st);
    timing_end(s, st);
    if (rc != CLOTH_OK) return rc;
    rc = toi_merge_filter(s, c, xm, xp, dxo, st);
    if (rc == CLOTH_OK && setup) rc = block_setup(s, c, st);
    timing_end(s, st);
    return rc;
}

cloth_status contact_step_begin(Scene& s, ContactState& c, const float* xp, hipStream_t st) {
    return outer_stage(s, c, s.d.xstar, xp, true, true, nullptr, st);
}

cloth_status contact_block_begin(Scene& s, ContactState& c, hipStream_t st) {
    (void)s;
    (void)c;
    (void)st;
    return CLOTH_OK;
}

cloth_status contact_block_end(Scene& s, ContactState& c, bool setup, unsigned long long* dxo, hipStream_t st) {
    return outer_stage(s, c, s.d.xm, s.d.xk, false, setup, dxo, st);
}

cloth_status contact_prepare_iteration(Scene& s, ContactState& c, bool force_k, hipStream_t st) {
    if (!s.self_contact) return CLOTH_OK;
    Dev& d = s.d;
    hipLaunchKernelGGL(k_pair_targets, dim3(cgrid(s, c)), dim3(TPB), 0, st, d, c.cnt, c.cpair, c.ca, c.clam,
                       c.cnrm, (float)s.kc, (float)s.Kb, (float)s.dhat, c.slot, force_k ? 1 : 0);
    HC(hipGetLastError());
    return CLOTH_OK;
}

cloth_status contact_build_uu(Scene& s) {
    if (!s.d.UU) return CLOTH_OK;
    const int grid = std::min(s.nv, 4096);
    if (s.prec == CLOTH_MIXED)
        hipLaunchKernelGGL(k_uu_build<uint16_t>, dim3(grid), dim3(256), 0, 0, s.d, s.d.UU);
    else
        hipLaunchKernelGGL(k_uu_build<float>, dim3(grid), dim3(256), 0, 0, s.d, s.d.UU);
    HC(hipGetLastError());
    HC(hipDeviceSynchronize());
    return CLOTH_OK;
}

// The contact matrix of the iteration (Eq. (subspace_collision) with the
// Gram of Eq. (uu)) and its factorization; it depends on the collision
// weights only, so it may run beside the local step (on a second stream).
cloth_status contact_factor(Scene& s, ContactState& c, bool force_k, hipStream_t st) {
    Dev& d = s.d;
    int* wchg = c.cnt + CNT_WCHG;
    // weights forced to k (residual forwarding) differ from the spans' ones;
    // friction weights follow the iterate, so they change every iteration
    if (force_k || (s.mu > 0 && !s.obst.empty()))
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, s.d.gate, wchg, 1, 1);
    const int tot = s.r * (s.r + 1) / 2;
    double* gred = d.Amat;
    double* Arm = d.Amat + (size_t)GRAM_GROUPS * tot;
    if (d.UU) {
        // Eq. (uu) from the precomputed store, straight into the group sums
        hipLaunchKernelGGL(k_uu_sum, dim3((tot + 255) / 256, GRAM_GROUPS), dim3(256), 0, st, d, c.cvlist,
                           c.cnt + 6, gred, (const int*)wchg, force_k ? 1 : 0);
    } else {
        const int T = (s.r + 15) / 16;   // 16 x 16 tiles per side of the Gram
        dim3 grid(c.gram_chunks, (T * (T + 1) / 2 + 4 * GRAM_TW - 1) / (4 * GRAM_TW));
        if (s.prec == CLOTH_MIXED)
            hipLaunchKernelGGL(k_gram<uint16_t>, grid, dim3(256), 0, st, d, c.cvlist, c.cnt + 6, c.gram_chunks,
                               d.gram_part, (const int*)wchg, force_k ? 1 : 0);
        else
            hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), 0, st, d, c.cvlist, c.cnt + 6, c.gram_chunks,
                               d.gram_part, (const int*)wchg, force_k ? 1 : 0);
        hipLaunchKernelGGL(k_gram_reduce, dim3((tot + 255) / 256, GRAM_GROUPS), dim3(256), 0, st, d, d.gram_part,
                           c.gram_chunks, c.cnt + 6, gred, (const int*)wchg);
    }
    hipLaunchKernelGGL(k_gram_final, dim3((tot + 255) / 256), dim3(256), 0, st, d, (const double*)gred, c.cnt + 6,
                       Arm, (const int*)wchg);
    hipLaunchKernelGGL(k_chol_factor, dim3(1), dim3(FT), chol_lds_bytes(s.r), st, d, (const double*)Arm,
                       (const int*)(c.cnt + 6), wchg, c.cnt + CNT_NFACT);
    HC(hipGetLastError());
    return CLOTH_OK;
}

// q = A^{-1} g on the factor of contact_factor; g = U^T r0 is in d.gvec
cloth_status contact_solve(Scene& s, ContactState& c, hipStream_t st) {
    Dev& d = s.d;
    const size_t lds = chol_lds_bytes(s.r) + sizeof(double) * 3 * s.r;
    if (s.r <= 128)
        hipLaunchKernelGGL(k_chol_tri<2>, dim3(1), dim3(1024), lds, st, d, (const int*)(c.cnt + 6));
    else
        hipLaunchKernelGGL(k_chol_tri<3>, dim3(1), dim3(1024), lds, st, d, (const int*)(c.cnt + 6));
    HC(hipGetLastError());
    return CLOTH_OK;
}

cloth_status contact_partial_ccd(Scene& s, ContactState& c, hipStream_t st, bool targets) {
    Dev& d = s.d;
    const bool tg = targets && s.self_contact;
    hipLaunchKernelGGL(k_partial_ccd, dim3(std::min(gblocks(2 * c.cap + s.nv), gblocks(2 * (int64_t)s.nv))), dim3(TPB), 0, st, d, c.cnt, c.cpair, c.ca,
                       c.clam, s.amax, d.xk, c.cnt + CNT_WCHG, s.adapt_samples, tg ? 1 : 0, (const float4*)c.cnrm,
                       (float)s.kc, (float)s.Kb, (float)s.dhat, c.slot);
    HC(hipGetLastError());
    return CLOTH_OK;
}

cloth_status contact_reset(Scene& s, ContactState& c, hipStream_t st) {
    (void)s;
    if (c.cnt) {
        HC(hipMemsetAsync(c.cnt + CNT_STEP_FAIL, 0, sizeof(int), st));
        HC(hipMemsetAsync(c.cnt + PEAK_SLOT, 0, sizeof(int), st));
        HC(hipMemsetAsync(c.cnt + CNT_STICKY, 0, 2 * sizeof(int), st));
    }
    return CLOTH_OK;
}

cloth_status contact_stats(Scene& s, ContactState& c, hipStream_t st, cloth_step_stats* out) {
    if (!c.enabled) return CLOTH_OK;
    int h[CNT_WORDS];
    unsigned long long tb[2];
    HC(hipMemcpyAsync(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    HC(hipMemcpyAsync(tb, c.tmin_bits, sizeof(tb), hipMemcpyDeviceToHost, st));
    HC(hipStreamSynchronize(st));
    double t;
    std::memcpy(&t, &tb[1], 8);
    out->min_toi = t;
    out->n_candidates = (int64_t)h[0] + h[1];
    out->n_constraints = (int64_t)h[2] + h[3] + h[10];
    out->peak_candidates = h[12];
    out->n_contact_vertices = h[6];
    out->n_factorizations = h[CNT_NFACT];
    int sw[8];
    HC(hipMemcpyAsync(sw, c.supw, sizeof(sw), hipMemcpyDeviceToHost, st));
    HC(hipStreamSynchronize(st));
    out->n_broad_rebuilds = sw[3];
    HC(hipMemsetAsync(c.supw + 3, 0, sizeof(int), st));
    HC(hipMemsetAsync(c.cnt + 12, 0, sizeof(int), st));
    HC(hipMemsetAsync(c.cnt + CNT_NFACT, 0, sizeof(int), st));
    (void)s;
    return CLOTH_OK;
}

// text for the status bits of a failed step
std::string step_failure_text(const Scene& s, const ContactState& c, int bits) {
    std::string why;
    if (bits & OVF_QUERY) why += " a broad-phase query exceeded its work bound (cells, records or pairs);";
    if (bits & OVF_CELL) why += " a box could not be placed on the broad-phase grid;";
    if (bits & OVF_LIST) why += " a candidate list exceeded the pair capacity (" + std::to_string(c.cap) + ");";
    if (bits & OVF_CONS) why += " the constraint set exceeded its capacity (" + std::to_string(c.ccap) + ");";
    if (bits & STEP_DIVERGED) why += " an iterate became non-finite;";
    if (bits & STEP_TANGLED) why += " the tangle check found edges crossing triangles;";
    (void)s;
    return why;
}

// ---- stage entry points (host arrays, caller order; SoA conversion here)

static void to_soa(const float* a, std::vector<float>& o, int n) {
    o.resize(3 * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) o[(size_t)k * n + i] = a[3 * (size_t)i + k];
}

cloth_status contact_stage_broad_phase(Scene& s, ContactState& c, const float* xm, const float* xp, int64_t cap,
                                       int32_t* vt, int64_t* n_vt, int32_t* ee, int64_t* n_ee) {
    if (!s.self_contact) {
        *n_vt = *n_ee = 0;
        return CLOTH_OK;
    }
    std::vector<float> t;
    to_soa(xm, t, s.nv);
    HC(hipMemcpy(s.d.xm, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    to_soa(xp, t, s.nv);
    HC(hipMemcpy(s.d.xt, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_stage_counters, dim3(1), dim3(64), 0, nullptr, s.d.gate, c.cnt, 1, c.tmin_bits);
    HC(hipMemset(c.cnt + 7, 0, sizeof(int)));
    cloth_status rc = broad_phase(s, c, s.d.xm, s.d.xt, nullptr);
    if (rc != CLOTH_OK) return rc;
    int h[16];
    HC(hipMemcpy(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost));
    *n_vt = h[0];
    *n_ee = h[1];
    if (h[7]) HC(hipMemset(c.cnt + 7, 0, sizeof(int)));
    if (h[7] || h[0] > cap || h[1] > cap) return set_error(CLOTH_E_CAPACITY, "pair list does not fit");
    if (vt && h[0]) HC(hipMemcpy(vt, c.cand_vt, sizeof(int2) * h[0], hipMemcpyDeviceToHost));
    if (ee && h[1]) HC(hipMemcpy(ee, c.cand_ee, sizeof(int2) * h[1], hipMemcpyDeviceToHost));
    return CLOTH_OK;
}

cloth_status contact_stage_toi(Scene& s, ContactState& c, const float* xm, const float* xp, int64_t n_vt,
                               const int32_t* vt, int64_t n_ee, const int32_t* ee, double* toi_vt, double* toi_ee) {
    if (!s.self_contact) return set_error(CLOTH_E_INVALID, "pair TOI needs a scene with self contact");
    if (n_vt > c.cap || n_ee > c.cap) return set_error(CLOTH_E_CAPACITY, "pair list exceeds capacity");
    std::vector<float> t;
    to_soa(xm, t, s.nv);
    HC(hipMemcpy(s.d.xm, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    to_soa(xp, t, s.nv);
    HC(hipMemcpy(s.d.xt, t.data(), 12 * (size_t)s.nv, hipMemcpyHostToDevice));
    if (n_vt) HC(hipMemcpy(c.cand_vt, vt, sizeof(int2) * n_vt, hipMemcpyHostToDevice));
    if (n_ee) HC(hipMemcpy(c.cand_ee, ee, sizeof(int2) * n_ee, hipMemcpyHostToDevice));
    int h[2] = {(int)n_vt, (int)n_ee};
    HC(hipMemcpy(c.cnt, h, sizeof(h), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_aos4, dim3(gblocks(s.nv)), dim3(TPB), 0, nullptr, s.nv, (const float*)s.d.xm, c.xm4);
    hipLaunchKernelGGL(k_aos4, dim3(gblocks(s.nv)), dim3(TPB), 0, nullptr, s.nv, (const float*)s.d.xt, c.xp4);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, nullptr, s.d.gate, c.toi_sched, 0, 8 * TOI_LINE);
    hipLaunchKernelGGL(k_toi_merge, dim3(gblocks(n_vt + n_ee)), dim3(TPB), 0, nullptr, s.d, (const float4*)c.xm4,
                       (const float4*)c.xp4, c.cand_vt, c.cand_ee, c.cnt, c.toi_vt, c.toi_ee, c.keep, c.cand_a,
                       c.tpart, 0, c.toi_sched);
    HC(hipGetLastError());
    HC(hipDeviceSynchronize());
    if (n_vt) HC(hipMemcpy(toi_vt, c.toi_vt, sizeof(double) * n_vt, hipMemcpyDeviceToHost));
    if (n_ee) HC(hipMemcpy(toi_ee, c.toi_ee, sizeof(double) * n_ee, hipMemcpyDeviceToHost));
    return CLOTH_OK;
}

cloth_status contact_load_constraints(Scene& s, ContactState& c, int64_t n_vt, const int32_t* vt, const int32_t* a_vt,
                                      int64_t n_ee, const int32_t* ee, const int32_t* a_ee, const int32_t* ob_a) {
    const int n = s.nv;
    if (!c.enabled) {
        c.active = false;
        return CLOTH_OK;
    }
    if (n_vt + n_ee > c.ccap) return set_error(CLOTH_E_CAPACITY, "constraint list exceeds capacity");
    if ((n_vt || n_ee) && !s.self_contact) return set_error(CLOTH_E_INVALID, "pair constraints without self contact");
    std::vector<int2> pr(n_vt + n_ee);
    std::vector<int> a(n_vt + n_ee);
    for (int64_t i = 0; i < n_vt; ++i) {
        pr[i] = make_int2(vt[2 * i], vt[2 * i + 1]);
        a[i] = a_vt ? a_vt[i] : 0;
    }
    for (int64_t i = 0; i < n_ee; ++i) {
        pr[n_vt + i] = make_int2(ee[2 * i], ee[2 * i + 1]);
        a[n_vt + i] = a_ee ? a_ee[i] : 0;
    }
    if (!pr.empty()) {
        HC(hipMemcpy(c.cpair, pr.data(), sizeof(int2) * pr.size(), hipMemcpyHostToDevice));
        HC(hipMemcpy(c.ca, a.data(), sizeof(int) * a.size(), hipMemcpyHostToDevice));
    }
    int h[16] = {0};
    h[2] = (int)n_vt;
    h[3] = (int)n_ee;
    HC(hipMemcpy(c.cnt, h, sizeof(h), hipMemcpyHostToDevice));
    std::vector<int> ob(MAX_OBST * (size_t)n, -1);
    if (ob_a)
        for (int j = 0; j < c.nob; ++j)
            for (int v = 0; v < n; ++v) ob[(size_t)j * n + v] = ob_a[(size_t)j * n + v];
    HC(hipMemcpy(c.ob_a, ob.data(), sizeof(int) * ob.size(), hipMemcpyHostToDevice));
    return block_setup(s, c, nullptr);
}

cloth_status contact_read_constraints(Scene& s, ContactState& c, int32_t* a_vt, int32_t* a_ee, int32_t* ob_a) {
    if (!c.enabled) return CLOTH_OK;
    int h[16];
    HC(hipMemcpy(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost));
    if (a_vt && h[2]) HC(hipMemcpy(a_vt, c.ca, sizeof(int) * h[2], hipMemcpyDeviceToHost));
    if (a_ee && h[3]) HC(hipMemcpy(a_ee, c.ca + h[2], sizeof(int) * h[3], hipMemcpyDeviceToHost));
    if (ob_a && c.nob)
        HC(hipMemcpy(ob_a, c.ob_a, sizeof(int) * (size_t)c.nob * s.nv, hipMemcpyDeviceToHost));
    return CLOTH_OK;
}

cloth_status contact_stage_outer(Scene& s, ContactState& c, const float* xm, const float* xp, int first,
                                 float* x_out, double* s_out) {
    if (!c.enabled) return set_error(CLOTH_E_INVALID, "no contact in this scene");
    const int n = s.nv;
    std::vector<float> t;
    to_soa(xm, t, n);
    HC(hipMemcpy(s.d.xm, t.data(), 12 * (size_t)n, hipMemcpyHostToDevice));
    to_soa(xp, t, n);
    HC(hipMemcpy(s.d.xt, t.data(), 12 * (size_t)n, hipMemcpyHostToDevice));
    HC(hipMemset(c.cnt + 7, 0, sizeof(int)));
    cloth_status rc = outer_stage(s, c, s.d.xm, s.d.xt, first != 0, true, nullptr, nullptr);
    if (rc != CLOTH_OK) return rc;
    HC(hipDeviceSynchronize());
    int h[16];
    HC(hipMemcpy(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost));
    if (h[7]) {
        HC(hipMemset(c.cnt + 7, 0, sizeof(int)));
        return set_error(CLOTH_E_CAPACITY, "pair capacity exceeded");
    }
    if (s_out) HC(hipMemcpy(s_out, c.s_dev, 8, hipMemcpyDeviceToHost));
    if (x_out) {
        HC(hipMemcpy(t.data(), s.d.x, 12 * (size_t)n, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) x_out[3 * (size_t)i + k] = t[(size_t)k * n + i];
    }
    return CLOTH_OK;
}

cloth_status contact_stage_read_set(Scene& s, ContactState& c, int64_t cap, int32_t* vt, int32_t* a_vt,
                                    int64_t* n_vt, int32_t* ee, int32_t* a_ee, int64_t* n_ee, int32_t* ob_a) {
    int h[16];
    HC(hipMemcpy(h, c.cnt, sizeof(h), hipMemcpyDeviceToHost));
    if (n_vt) *n_vt = h[2];
    if (n_ee) *n_ee = h[3];
    int64_t mv = std::min<int64_t>(h[2], cap), me = std::min<int64_t>(h[3], cap);
    if (vt && mv) HC(hipMemcpy(vt, c.cpair, sizeof(int2) * mv, hipMemcpyDeviceToHost));
    if (a_vt && mv) HC(hipMemcpy(a_vt, c.ca, sizeof(int) * mv, hipMemcpyDeviceToHost));
    if (ee && me) HC(hipMemcpy(ee, c.cpair + h[2], sizeof(int2) * me, hipMemcpyDeviceToHost));
    if (a_ee && me) HC(hipMemcpy(a_ee, c.ca + h[2], sizeof(int) * me, hipMemcpyDeviceToHost));
    if (ob_a && c.nob) HC(hipMemcpy(ob_a, c.ob_a, sizeof(int) * (size_t)c.nob * s.nv, hipMemcpyDeviceToHost));
    if (h[2] > cap || h[3] > cap) return set_error(CLOTH_E_CAPACITY, "constraint list does not fit");
    return CLOTH_OK;
}

void contact_destroy(Scene& s, ContactState& c) {
    (void)s;
    (void)c;
}

}  // namespace cloth
