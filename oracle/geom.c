/*
 * Oracle geometry (TEST INFRASTRUCTURE ONLY — never linked into the library).
 *
 * Plain, slow, FP64 C for the collision side of the cloth solver:
 *   - broad phase: every vertex-triangle (VT) and edge-edge (EE) pair whose
 *     swept, inflated FP32 boxes overlap (exact box tests, results sorted);
 *   - full CCD: earliest time in [0,1] at which a VT/EE pair is coplanar (a
 *     cubic in t) and in contact (inside test), with a sampled fallback for
 *     degenerate cubics (paper section 4.1 and 8.1: exact TOI per pair);
 *   - closest points at the start of an outer block (frozen constraint data);
 *   - a triangle-triangle intersection count (tangle check) with a filtered
 *     orientation predicate that hands uncertain cases back to the caller.
 *
 * Compiled with -O2 -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 crs(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 ldp(const float* x, int i) { return mk((double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]); }
static v3 ldd(const double* x, int i) { return mk(x[3 * i], x[3 * i + 1], x[3 * i + 2]); }
static v3 lerp(v3 a, v3 b, double t) { return add(a, scl(sub(b, a), t)); }
static double amax3(v3 a) {
    double m = fabs(a.x);
    if (fabs(a.y) > m) m = fabs(a.y);
    if (fabs(a.z) > m) m = fabs(a.z);
    return m;
}

/* ------------------------------------------------------------------ boxes */

typedef struct { float lo[3], hi[3]; } box;

static box swept_box(const float* xm, const float* xp, const int* v, int nvert, float dhat) {
    box b;
    for (int d = 0; d < 3; ++d) {
        float lo = xm[3 * v[0] + d], hi = lo;
        for (int k = 0; k < nvert; ++k) {
            float a = xm[3 * v[k] + d], c = xp[3 * v[k] + d];
            if (a < lo) lo = a;
            if (a > hi) hi = a;
            if (c < lo) lo = c;
            if (c > hi) hi = c;
        }
        b.lo[d] = lo - dhat;
        b.hi[d] = hi + dhat;
    }
    return b;
}

static int overlap(const box* a, const box* b) {
    for (int d = 0; d < 3; ++d)
        if (a->lo[d] > b->hi[d] || b->lo[d] > a->hi[d]) return 0;
    return 1;
}

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* A 2-D (x, z) bucket grid: each "target" box is filed in the one cell that
 * holds its low corner; a query scans every cell whose range could hold the
 * low corner of an overlapping box (low corner within [qlo - maxw, qhi]).
 * Every target is therefore visited at most once per query, and every
 * overlapping target is visited. */
typedef struct {
    int nx, nz;
    double ox, oz, cell;
    int* start; /* nx*nz+1 */
    int* items;
} grid2;

static void grid_build(grid2* g, const box* bx, int n, float maxw) {
    double mnx = 1e300, mnz = 1e300, mxx = -1e300, mxz = -1e300;
    for (int i = 0; i < n; ++i) {
        if (bx[i].lo[0] < mnx) mnx = bx[i].lo[0];
        if (bx[i].lo[2] < mnz) mnz = bx[i].lo[2];
        if (bx[i].lo[0] > mxx) mxx = bx[i].lo[0];
        if (bx[i].lo[2] > mxz) mxz = bx[i].lo[2];
    }
    if (n == 0) { mnx = mnz = 0; mxx = mxz = 1; }
    double cell = maxw > 0 ? maxw : 1.0;
    double ext = (mxx - mnx) > (mxz - mnz) ? (mxx - mnx) : (mxz - mnz);
    if (ext / cell > 4096.0) cell = ext / 4096.0;
    g->cell = cell;
    g->ox = mnx;
    g->oz = mnz;
    g->nx = (int)floor((mxx - mnx) / cell) + 1;
    g->nz = (int)floor((mxz - mnz) / cell) + 1;
    int nc = g->nx * g->nz;
    g->start = (int*)calloc((size_t)nc + 1, sizeof(int));
    g->items = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int* cid = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        int ix = (int)floor((bx[i].lo[0] - g->ox) / cell);
        int iz = (int)floor((bx[i].lo[2] - g->oz) / cell);
        if (ix < 0) ix = 0;
        if (iz < 0) iz = 0;
        if (ix >= g->nx) ix = g->nx - 1;
        if (iz >= g->nz) iz = g->nz - 1;
        cid[i] = ix * g->nz + iz;
        g->start[cid[i] + 1]++;
    }
    for (int c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
    int* fill = (int*)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    memcpy(fill, g->start, sizeof(int) * (size_t)nc);
    for (int i = 0; i < n; ++i) g->items[fill[cid[i]]++] = i;
    free(fill);
    free(cid);
}

static void grid_free(grid2* g) {
    free(g->start);
    free(g->items);
}

static void grid_range(const grid2* g, double lo, double hi, double o, int nmax, int* a, int* b) {
    int i0 = (int)floor((lo - o) / g->cell) - 1;
    int i1 = (int)floor((hi - o) / g->cell) + 1;
    if (i0 < 0) i0 = 0;
    if (i1 > nmax - 1) i1 = nmax - 1;
    *a = i0;
    *b = i1;
}

static float max_width(const box* bx, int n) {
    float w = 0;
    for (int i = 0; i < n; ++i) {
        if (bx[i].hi[0] - bx[i].lo[0] > w) w = bx[i].hi[0] - bx[i].lo[0];
        if (bx[i].hi[2] - bx[i].lo[2] > w) w = bx[i].hi[2] - bx[i].lo[2];
    }
    return w;
}

/* Candidate pairs.  VT pairs (v, t) with v not a corner of t, EE pairs
 * (e1, e2) with e1 < e2 sharing no vertex; boxes are swept over (xm, xp) and
 * grown by dhat on every side, all in FP32.  Output sorted by (first, second).
 * Returns 0, or -1 if a capacity was exceeded (the counts then hold the
 * number of pairs that exist). */
int og_broad_phase(int nv, const float* xm, const float* xp, int ne, const int* edges, int nt,
                   const int* tris, float dhat, int self_contact, long cap_vt, int* vt_out,
                   long* n_vt, long cap_ee, int* ee_out, long* n_ee) {
    *n_vt = 0;
    *n_ee = 0;
    if (!self_contact) return 0;
    box* bv = (box*)malloc(sizeof(box) * (size_t)(nv > 0 ? nv : 1));
    box* bt = (box*)malloc(sizeof(box) * (size_t)(nt > 0 ? nt : 1));
    box* be = (box*)malloc(sizeof(box) * (size_t)(ne > 0 ? ne : 1));
    for (int v = 0; v < nv; ++v) bv[v] = swept_box(xm, xp, &v, 1, dhat);
    for (int t = 0; t < nt; ++t) bt[t] = swept_box(xm, xp, tris + 3 * t, 3, dhat);
    for (int e = 0; e < ne; ++e) be[e] = swept_box(xm, xp, edges + 2 * e, 2, dhat);
    int rc = 0;
    int* buf = (int*)malloc(sizeof(int) * (size_t)(nt + ne + 1));

    /* VT */
    {
        float wt = max_width(bt, nt);
        grid2 g;
        grid_build(&g, bt, nt, wt);
        for (int v = 0; v < nv; ++v) {
            int cnt = 0, x0, x1, z0, z1;
            grid_range(&g, bv[v].lo[0] - wt, bv[v].hi[0], g.ox, g.nx, &x0, &x1);
            grid_range(&g, bv[v].lo[2] - wt, bv[v].hi[2], g.oz, g.nz, &z0, &z1);
            for (int ix = x0; ix <= x1; ++ix)
                for (int iz = z0; iz <= z1; ++iz) {
                    int c = ix * g.nz + iz;
                    for (int k = g.start[c]; k < g.start[c + 1]; ++k) {
                        int t = g.items[k];
                        const int* tv = tris + 3 * t;
                        if (tv[0] == v || tv[1] == v || tv[2] == v) continue;
                        if (overlap(&bv[v], &bt[t])) buf[cnt++] = t;
                    }
                }
            qsort(buf, (size_t)cnt, sizeof(int), cmp_int);
            for (int k = 0; k < cnt; ++k) {
                if (*n_vt < cap_vt) {
                    vt_out[2 * *n_vt] = v;
                    vt_out[2 * *n_vt + 1] = buf[k];
                } else {
                    rc = -1;
                }
                (*n_vt)++;
            }
        }
        grid_free(&g);
    }
    /* EE */
    {
        float we = max_width(be, ne);
        grid2 g;
        grid_build(&g, be, ne, we);
        for (int e = 0; e < ne; ++e) {
            int cnt = 0, x0, x1, z0, z1;
            const int* a = edges + 2 * e;
            grid_range(&g, be[e].lo[0] - we, be[e].hi[0], g.ox, g.nx, &x0, &x1);
            grid_range(&g, be[e].lo[2] - we, be[e].hi[2], g.oz, g.nz, &z0, &z1);
            for (int ix = x0; ix <= x1; ++ix)
                for (int iz = z0; iz <= z1; ++iz) {
                    int c = ix * g.nz + iz;
                    for (int k = g.start[c]; k < g.start[c + 1]; ++k) {
                        int f = g.items[k];
                        if (f <= e) continue;
                        const int* b = edges + 2 * f;
                        if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
                        if (overlap(&be[e], &be[f])) buf[cnt++] = f;
                    }
                }
            qsort(buf, (size_t)cnt, sizeof(int), cmp_int);
            for (int k = 0; k < cnt; ++k) {
                if (*n_ee < cap_ee) {
                    ee_out[2 * *n_ee] = e;
                    ee_out[2 * *n_ee + 1] = buf[k];
                } else {
                    rc = -1;
                }
                (*n_ee)++;
            }
        }
        grid_free(&g);
    }
    free(buf);
    free(bv);
    free(bt);
    free(be);
    return rc;
}

/* ------------------------------------------------------------ full CCD */

#define CCD_DEGEN_REL 1e-14   /* cubic treated as identically zero below this x L^3 */
#define CCD_PAR_REL 1e-20     /* edges parallel when sin^2(angle) below this */
#define CCD_SAMPLES 1024      /* time samples of the degenerate fallback */
#define NO_HIT 2.0

static double horner(const double c[4], double t) { return ((c[3] * t + c[2]) * t + c[1]) * t + c[0]; }

static int sgn(double v) { return (v > 0) - (v < 0); }

/* Roots of the cubic c in [0,1], ascending; returns their number.  The
 * interval is split at the roots of the derivative, and every piece whose end
 * values have opposite signs (or a zero end) is bisected 64 times; the low end
 * of the final bracket is the root (never past the crossing). */
static int cubic_roots01(const double c[4], double* roots) {
    double brk[4];
    int nb = 0;
    brk[nb++] = 0.0;
    /* derivative 3 c3 t^2 + 2 c2 t + c1 */
    double A = 3 * c[3], B = 2 * c[2], C = c[1];
    double cr[2];
    int ncr = 0;
    if (A != 0.0) {
        double disc = B * B - 4 * A * C;
        if (disc >= 0) {
            double sq = sqrt(disc);
            double q = -0.5 * (B + (B >= 0 ? sq : -sq));
            double r1 = q / A, r2 = (q != 0.0) ? C / q : r1;
            if (r1 > r2) { double tt = r1; r1 = r2; r2 = tt; }
            cr[ncr++] = r1;
            if (r2 != r1) cr[ncr++] = r2;
        }
    } else if (B != 0.0) {
        cr[ncr++] = -C / B;
    }
    for (int i = 0; i < ncr; ++i)
        if (cr[i] > 0.0 && cr[i] < 1.0) brk[nb++] = cr[i];
    brk[nb++] = 1.0;
    int nr = 0;
    for (int i = 0; i + 1 < nb; ++i) {
        double lo = brk[i], hi = brk[i + 1];
        double flo = horner(c, lo), fhi = horner(c, hi);
        if (flo == 0.0) {
            if (nr == 0 || roots[nr - 1] != lo) roots[nr++] = lo;
            continue;
        }
        if (fhi == 0.0) {
            roots[nr++] = hi;
            continue;
        }
        if (sgn(flo) == sgn(fhi)) continue;
        int s0 = sgn(flo);
        for (int it = 0; it < 64; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double fm = horner(c, mid);
            if (fm == 0.0) { lo = mid; break; }
            if (sgn(fm) == s0) lo = mid; else hi = mid;
        }
        roots[nr++] = lo;
    }
    return nr;
}

/* Closed point-in-triangle test for p in (or near) the plane of abc. */
static int inside_tri(v3 p, v3 a, v3 b, v3 c) {
    v3 n = crs(sub(b, a), sub(c, a));
    if (dot(n, n) <= 0.0) return 0;
    double u = dot(crs(sub(b, p), sub(c, p)), n);
    double v = dot(crs(sub(c, p), sub(a, p)), n);
    double w = dot(crs(sub(a, p), sub(b, p)), n);
    return u >= 0.0 && v >= 0.0 && w >= 0.0;
}

/* Closed segment-segment crossing test for coplanar segments p1p2, p3p4;
 * returns -1 when the segments are (numerically) parallel. */
static int cross_seg(v3 p1, v3 p2, v3 p3, v3 p4) {
    v3 d1 = sub(p2, p1), d2 = sub(p4, p3), r = sub(p3, p1);
    v3 n = crs(d1, d2);
    double nn = dot(n, n);
    if (nn <= CCD_PAR_REL * dot(d1, d1) * dot(d2, d2)) return -1;
    double s1 = dot(crs(r, d2), n) / nn;
    double s2 = dot(crs(r, d1), n) / nn;
    return s1 >= 0.0 && s1 <= 1.0 && s2 >= 0.0 && s2 <= 1.0;
}

/* Point-triangle and segment-segment distances (for the fallback). */
static void closest_on_tri(v3 p, v3 a, v3 b, v3 c, double* l1, double* l2);
static void closest_seg_seg(v3 p1, v3 p2, v3 p3, v3 p4, double* s, double* t);

static double dist_pt_tri(v3 p, v3 a, v3 b, v3 c) {
    double l1, l2;
    closest_on_tri(p, a, b, c, &l1, &l2);
    v3 q = add(a, add(scl(sub(b, a), l1), scl(sub(c, a), l2)));
    v3 d = sub(p, q);
    return sqrt(dot(d, d));
}

static double dist_seg_seg(v3 p1, v3 p2, v3 p3, v3 p4) {
    double s, t;
    closest_seg_seg(p1, p2, p3, p4, &s, &t);
    v3 d = sub(lerp(p3, p4, t), lerp(p1, p2, s));
    return sqrt(dot(d, d));
}

/* Degenerate fallback: first of CCD_SAMPLES+1 uniform times at which the
 * distance is at most eta, refined by 64 bisections on that predicate. */
typedef double (*distfn)(const v3* p0, const v3* p1, double t);

static double d_vt(const v3* p0, const v3* p1, double t) {
    return dist_pt_tri(lerp(p0[0], p1[0], t), lerp(p0[1], p1[1], t), lerp(p0[2], p1[2], t),
                       lerp(p0[3], p1[3], t));
}
static double d_ee(const v3* p0, const v3* p1, double t) {
    return dist_seg_seg(lerp(p0[0], p1[0], t), lerp(p0[1], p1[1], t), lerp(p0[2], p1[2], t),
                        lerp(p0[3], p1[3], t));
}

static double sampled_toi(const v3* p0, const v3* p1, distfn f, double eta) {
    double prev = 0.0;
    for (int i = 0; i <= CCD_SAMPLES; ++i) {
        double t = (double)i / CCD_SAMPLES;
        if (f(p0, p1, t) <= eta) {
            if (i == 0) return 0.0;
            double lo = prev, hi = t;
            for (int it = 0; it < 64; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (f(p0, p1, mid) <= eta) hi = mid; else lo = mid;
            }
            return lo;
        }
        prev = t;
    }
    return NO_HIT;
}

/* Coefficients of f(t) = ((b-a) x (c-a)) . (p-a) along linear motion, for
 * the four moving points q[0..3] = (p, a, b, c) or (p1, p2, p3, p4) mapped to
 * the same form. Also returns L, the largest relative coordinate used. */
static void coplanar_cubic(const v3* q0, const v3* q1, double c[4], double* L) {
    /* relative to q[1] */
    v3 E1 = sub(q0[2], q0[1]), E2 = sub(q0[3], q0[1]), W = sub(q0[0], q0[1]);
    v3 F1 = sub(q1[2], q1[1]), F2 = sub(q1[3], q1[1]), Wf = sub(q1[0], q1[1]);
    v3 dE1 = sub(F1, E1), dE2 = sub(F2, E2), dW = sub(Wf, W);
    v3 C0 = crs(E1, E2);
    v3 C1 = add(crs(E1, dE2), crs(dE1, E2));
    v3 C2 = crs(dE1, dE2);
    c[0] = dot(C0, W);
    c[1] = dot(C0, dW) + dot(C1, W);
    c[2] = dot(C1, dW) + dot(C2, W);
    c[3] = dot(C2, dW);
    double m = 0;
    v3 all[6] = {E1, E2, W, F1, F2, Wf};
    for (int i = 0; i < 6; ++i)
        if (amax3(all[i]) > m) m = amax3(all[i]);
    *L = m;
}

static int degenerate(const double c[4], double L) {
    double s = fabs(c[0]);
    for (int i = 1; i < 4; ++i)
        if (fabs(c[i]) > s) s = fabs(c[i]);
    return s <= CCD_DEGEN_REL * L * L * L;
}

/* VT time of impact: vertex p moving p0->p1, triangle (a,b,c). */
double og_toi_vt(const double* P0, const double* P1, int* used_fallback) {
    v3 q0[4], q1[4];
    for (int k = 0; k < 4; ++k) {
        q0[k] = mk(P0[3 * k], P0[3 * k + 1], P0[3 * k + 2]);
        q1[k] = mk(P1[3 * k], P1[3 * k + 1], P1[3 * k + 2]);
    }
    double c[4], L;
    coplanar_cubic(q0, q1, c, &L);
    *used_fallback = 0;
    if (L == 0.0) return NO_HIT;
    if (degenerate(c, L)) {
        *used_fallback = 1;
        return sampled_toi(q0, q1, d_vt, 1e-12 * L);
    }
    double roots[4];
    int nr = cubic_roots01(c, roots);
    for (int i = 0; i < nr; ++i) {
        double t = roots[i];
        if (inside_tri(lerp(q0[0], q1[0], t), lerp(q0[1], q1[1], t), lerp(q0[2], q1[2], t),
                       lerp(q0[3], q1[3], t)))
            return t;
    }
    return NO_HIT;
}

/* EE time of impact: edges (p1,p2) and (p3,p4); f(t) = (p2-p1)x(p4-p3).(p3-p1). */
double og_toi_ee(const double* P0, const double* P1, int* used_fallback) {
    v3 e0[4], e1[4];
    for (int k = 0; k < 4; ++k) {
        e0[k] = mk(P0[3 * k], P0[3 * k + 1], P0[3 * k + 2]);
        e1[k] = mk(P1[3 * k], P1[3 * k + 1], P1[3 * k + 2]);
    }
    /* map to the VT form: "p" = p3, "a" = p1, "b" = p2, "c" = p1 + (p4 - p3).
     * (b-a) x (c-a) . (p-a) = (p2-p1) x (p4-p3) . (p3-p1). */
    v3 q0[4] = {e0[2], e0[0], e0[1], add(e0[0], sub(e0[3], e0[2]))};
    v3 q1[4] = {e1[2], e1[0], e1[1], add(e1[0], sub(e1[3], e1[2]))};
    double c[4], L;
    coplanar_cubic(q0, q1, c, &L);
    *used_fallback = 0;
    if (L == 0.0) return NO_HIT;
    if (degenerate(c, L)) {
        *used_fallback = 1;
        return sampled_toi(e0, e1, d_ee, 1e-12 * L);
    }
    double roots[4];
    int nr = cubic_roots01(c, roots);
    for (int i = 0; i < nr; ++i) {
        double t = roots[i];
        int r = cross_seg(lerp(e0[0], e1[0], t), lerp(e0[1], e1[1], t), lerp(e0[2], e1[2], t),
                          lerp(e0[3], e1[3], t));
        if (r < 0) {
            *used_fallback = 1;
            return sampled_toi(e0, e1, d_ee, 1e-12 * L);
        }
        if (r) return t;
    }
    return NO_HIT;
}

/* Batched TOI over candidate lists (FP32 positions promoted to FP64). */
void og_toi_pairs(const double* xm, const double* xp, const int* tris, const int* edges, long n_vt,
                  const int* vt, long n_ee, const int* ee, double* toi_vt, double* toi_ee,
                  long* n_fallback) {
    long nf = 0;
    for (long i = 0; i < n_vt; ++i) {
        int v = vt[2 * i], t = vt[2 * i + 1];
        int id[4] = {v, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        double P0[12], P1[12];
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) {
                P0[3 * k + d] = xm[3 * id[k] + d];
                P1[3 * k + d] = xp[3 * id[k] + d];
            }
        int fb;
        toi_vt[i] = og_toi_vt(P0, P1, &fb);
        nf += fb;
    }
    for (long i = 0; i < n_ee; ++i) {
        int a = ee[2 * i], b = ee[2 * i + 1];
        int id[4] = {edges[2 * a], edges[2 * a + 1], edges[2 * b], edges[2 * b + 1]};
        double P0[12], P1[12];
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) {
                P0[3 * k + d] = xm[3 * id[k] + d];
                P1[3 * k + d] = xp[3 * id[k] + d];
            }
        int fb;
        toi_ee[i] = og_toi_ee(P0, P1, &fb);
        nf += fb;
    }
    *n_fallback = nf;
}

/* ------------------------------------------------------- closest points */

/* Closest point of triangle abc to p, as (l1, l2) with q = a + l1 (b-a) + l2 (c-a).
 * Region test over the seven Voronoi regions of the triangle (three vertices,
 * three edges, the face), the published method of C. Ericson, Real-Time
 * Collision Detection (2005), sec. 5.1.5. */
static void closest_on_tri(v3 p, v3 a, v3 b, v3 c, double* l1, double* l2) {
    v3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0 && d2 <= 0) { *l1 = 0; *l2 = 0; return; }
    v3 bp = sub(p, b);
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0 && d4 <= d3) { *l1 = 1; *l2 = 0; return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) { *l1 = d1 / (d1 - d3); *l2 = 0; return; }
    v3 cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0 && d5 <= d6) { *l1 = 0; *l2 = 1; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) { *l1 = 0; *l2 = d2 / (d2 - d6); return; }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        *l1 = 1 - w;
        *l2 = w;
        return;
    }
    double den = va + vb + vc;
    if (den == 0.0) { *l1 = 0; *l2 = 0; return; }
    *l1 = vb / den;
    *l2 = vc / den;
}

static double clamp01(double v) { return v < 0 ? 0 : (v > 1 ? 1 : v); }

/* Closest points of segments p1p2 (parameter s) and p3p4 (parameter t):
 * minimise |p1 + s d1 - p3 - t d2|^2 over the unit square by the clamped
 * line-line solution of C. Ericson, Real-Time Collision Detection (2005),
 * sec. 5.1.9. */
static void closest_seg_seg(v3 p1, v3 p2, v3 p3, v3 p4, double* s_out, double* t_out) {
    v3 d1 = sub(p2, p1), d2 = sub(p4, p3), r = sub(p1, p3);
    double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    double s, t;
    if (a <= 0 && e <= 0) { *s_out = 0; *t_out = 0; return; }
    if (a <= 0) {
        s = 0;
        t = clamp01(f / e);
    } else {
        double c = dot(d1, r);
        if (e <= 0) {
            t = 0;
            s = clamp01(-c / a);
        } else {
            double b = dot(d1, d2);
            double den = a * e - b * b;
            s = den > 0 ? clamp01((b * f - c * e) / den) : 0.0;
            t = (b * s + f) / e;
            if (t < 0) {
                t = 0;
                s = clamp01(-c / a);
            } else if (t > 1) {
                t = 1;
                s = clamp01((b - c) / a);
            }
        }
    }
    *s_out = s;
    *t_out = t;
}

/* Frozen constraint data at the start of an outer block (positions xm):
 * VT rows out[4] = (l1, l2, n...) are written as
 *   lam[2*i..] = (l1, l2)  closest barycentric parameters,
 *   nrm[3*i..] = unit triangle normal times the side sign of the vertex.
 * EE rows: lam = (s, t) closest parameters, nrm = unit(p2 - p1) at the
 * closest points (fallback: unit(d1 x d2), then +y). */
void og_frozen_vt(const double* xm, const int* tris, long n, const int* vt, double* lam, double* nrm) {
    for (long i = 0; i < n; ++i) {
        int v = vt[2 * i], t = vt[2 * i + 1];
        v3 p = ldd(xm, v), a = ldd(xm, tris[3 * t]), b = ldd(xm, tris[3 * t + 1]), c = ldd(xm, tris[3 * t + 2]);
        double l1, l2;
        closest_on_tri(p, a, b, c, &l1, &l2);
        v3 n = crs(sub(b, a), sub(c, a));
        double nl = sqrt(dot(n, n));
        n = nl > 0 ? scl(n, 1.0 / nl) : mk(0, 1, 0);
        double side = dot(n, sub(p, a));
        if (side < 0) n = scl(n, -1.0);
        lam[2 * i] = l1;
        lam[2 * i + 1] = l2;
        nrm[3 * i] = n.x;
        nrm[3 * i + 1] = n.y;
        nrm[3 * i + 2] = n.z;
    }
}

void og_frozen_ee(const double* xm, const int* edges, long n, const int* ee, double* lam, double* nrm) {
    for (long i = 0; i < n; ++i) {
        int e = ee[2 * i], f = ee[2 * i + 1];
        v3 p1 = ldd(xm, edges[2 * e]), p2 = ldd(xm, edges[2 * e + 1]);
        v3 p3 = ldd(xm, edges[2 * f]), p4 = ldd(xm, edges[2 * f + 1]);
        double s, t;
        closest_seg_seg(p1, p2, p3, p4, &s, &t);
        v3 d = sub(lerp(p3, p4, t), lerp(p1, p2, s));
        double dl = sqrt(dot(d, d));
        v3 n;
        if (dl > 0) {
            n = scl(d, 1.0 / dl);
        } else {
            n = crs(sub(p2, p1), sub(p4, p3));
            double nl = sqrt(dot(n, n));
            n = nl > 0 ? scl(n, 1.0 / nl) : mk(0, 1, 0);
        }
        lam[2 * i] = s;
        lam[2 * i + 1] = t;
        nrm[3 * i] = n.x;
        nrm[3 * i + 1] = n.y;
        nrm[3 * i + 2] = n.z;
    }
}

/* ------------------------------------------------------------ tangles */

/* Sign of orient3d(a,b,c,d) = (b-a) x (c-a) . (d-a) with a static error
 * filter (the bound is a multiple of the evaluation's rounding-error bound);
 * returns +1/-1, 0 when every product of the expansion is exactly zero (the
 * FP32 inputs make their differences and a zero product exact, so the
 * determinant is exactly zero), or ORIENT_UNSURE when the FP64 value cannot
 * be trusted (the caller then decides exactly). */
#define ORIENT_UNSURE 2
static int orient_f(v3 a, v3 b, v3 c, v3 d) {
    v3 ab = sub(b, a), ac = sub(c, a), ad = sub(d, a);
    double det = ab.x * (ac.y * ad.z - ac.z * ad.y) - ab.y * (ac.x * ad.z - ac.z * ad.x) +
                 ab.z * (ac.x * ad.y - ac.y * ad.x);
    double perm = fabs(ab.x) * (fabs(ac.y * ad.z) + fabs(ac.z * ad.y)) +
                  fabs(ab.y) * (fabs(ac.x * ad.z) + fabs(ac.z * ad.x)) +
                  fabs(ab.z) * (fabs(ac.x * ad.y) + fabs(ac.y * ad.x));
    if (perm == 0.0) return 0;
    double eb = 1e-12 * perm;
    if (det > eb) return 1;
    if (det < -eb) return -1;
    return ORIENT_UNSURE;
}

/* Segment pq against triangle abc (closed), using filtered orientations.
 * Returns 1 = intersect, 0 = disjoint, -1 = undecided in FP64.  With the
 * endpoints strictly on both sides of the triangle's plane, the segment
 * meets the closed triangle iff the three edge orientations seen from pq
 * agree where they are not zero (a zero puts the crossing on that edge's
 * line). */
static int seg_tri(v3 p, v3 q, v3 a, v3 b, v3 c) {
    int s1 = orient_f(a, b, c, p), s2 = orient_f(a, b, c, q);
    if (s1 == ORIENT_UNSURE || s2 == ORIENT_UNSURE || s1 == 0 || s2 == 0) return -1;
    if (s1 == s2) return 0;
    int o[3] = {orient_f(p, q, a, b), orient_f(p, q, b, c), orient_f(p, q, c, a)};
    int sign = 0;
    for (int i = 0; i < 3; ++i) {
        if (o[i] == ORIENT_UNSURE) return -1;
        if (o[i] == 0) continue;
        if (sign != 0 && o[i] != sign) return 0;
        sign = o[i];
    }
    return 1;
}

/* Count intersecting pairs of vertex-disjoint triangles at positions x
 * (FP32 promoted exactly).  Pairs whose FP64 orientation signs are not
 * certain are returned in `undecided` (up to cap) for an exact re-check.
 * Returns the number of certain intersections. */
long og_tangles(int nv, const float* x, int nt, const int* tris, long cap, int* undecided,
                long* n_undecided, int* first_pair) {
    (void)nv;
    box* bt = (box*)malloc(sizeof(box) * (size_t)(nt > 0 ? nt : 1));
    for (int t = 0; t < nt; ++t) bt[t] = swept_box(x, x, tris + 3 * t, 3, 0.0f);
    float wt = max_width(bt, nt);
    grid2 g;
    grid_build(&g, bt, nt, wt);
    long hits = 0, und = 0;
    first_pair[0] = first_pair[1] = -1;
    for (int t = 0; t < nt; ++t) {
        const int* A = tris + 3 * t;
        int x0, x1, z0, z1;
        grid_range(&g, bt[t].lo[0] - wt, bt[t].hi[0], g.ox, g.nx, &x0, &x1);
        grid_range(&g, bt[t].lo[2] - wt, bt[t].hi[2], g.oz, g.nz, &z0, &z1);
        for (int ix = x0; ix <= x1; ++ix)
            for (int iz = z0; iz <= z1; ++iz) {
                int c = ix * g.nz + iz;
                for (int k = g.start[c]; k < g.start[c + 1]; ++k) {
                    int u = g.items[k];
                    if (u <= t) continue;
                    const int* B = tris + 3 * u;
                    int share = 0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) share |= (A[i] == B[j]);
                    if (share) continue;
                    if (!overlap(&bt[t], &bt[u])) continue;
                    v3 a0 = ldp(x, A[0]), a1 = ldp(x, A[1]), a2 = ldp(x, A[2]);
                    v3 b0 = ldp(x, B[0]), b1 = ldp(x, B[1]), b2 = ldp(x, B[2]);
                    int res[6] = {seg_tri(a0, a1, b0, b1, b2), seg_tri(a1, a2, b0, b1, b2),
                                  seg_tri(a2, a0, b0, b1, b2), seg_tri(b0, b1, a0, a1, a2),
                                  seg_tri(b1, b2, a0, a1, a2), seg_tri(b2, b0, a0, a1, a2)};
                    int any = 0, unk = 0;
                    for (int i = 0; i < 6; ++i) {
                        any |= (res[i] == 1);
                        unk |= (res[i] == -1);
                    }
                    if (any) {
                        if (hits == 0) { first_pair[0] = t; first_pair[1] = u; }
                        hits++;
                    } else if (unk) {
                        if (und < cap) {
                            undecided[2 * und] = t;
                            undecided[2 * und + 1] = u;
                        }
                        und++;
                    }
                }
            }
    }
    grid_free(&g);
    free(bt);
    *n_undecided = und;
    return hits;
}
