"""Exact triangle-triangle intersection decisions with integer arithmetic,
for the pairs whose FP64 orientation signs the C filter could not certify
(TEST INFRASTRUCTURE ONLY).

Every FP32 value is an integer multiple of 2^-149, so scaling all
coordinates by 2^149 turns them into Python integers exactly; the predicates
below only add, subtract, multiply and compare, and a common positive scale
leaves every sign they test unchanged."""
from __future__ import annotations

import numpy as np

from . import native

_FP32_SCALE_EXP = 149


def _exact_int(v) -> int:
    """The FP32 value v times 2^149, exactly."""
    num, den = float(np.float32(v)).as_integer_ratio()
    shift = _FP32_SCALE_EXP - (den.bit_length() - 1)
    return num << shift


def _orient(a, b, c, d) -> int:
    ab = [b[i] - a[i] for i in range(3)]
    ac = [c[i] - a[i] for i in range(3)]
    ad = [d[i] - a[i] for i in range(3)]
    det = (ab[0] * (ac[1] * ad[2] - ac[2] * ad[1]) - ab[1] * (ac[0] * ad[2] - ac[2] * ad[0])
           + ab[2] * (ac[0] * ad[1] - ac[1] * ad[0]))
    return (det > 0) - (det < 0)


def _seg_tri(p, q, a, b, c) -> bool:
    """Closed segment pq against closed triangle abc, exact."""
    s1, s2 = _orient(a, b, c, p), _orient(a, b, c, q)
    if s1 == 0 and s2 == 0:
        return _coplanar_seg_tri(p, q, a, b, c)
    if s1 == s2:
        return False
    o = [_orient(p, q, a, b), _orient(p, q, b, c), _orient(p, q, c, a)]
    nz = [v for v in o if v != 0]
    return all(v == nz[0] for v in nz) if nz else True


def _coplanar_seg_tri(p, q, a, b, c) -> bool:
    # project on the dominant plane of the triangle normal, then 2-D tests
    n = [(b[1] - a[1]) * (c[2] - a[2]) - (b[2] - a[2]) * (c[1] - a[1]),
         (b[2] - a[2]) * (c[0] - a[0]) - (b[0] - a[0]) * (c[2] - a[2]),
         (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])]
    drop = max(range(3), key=lambda i: abs(n[i]))
    keep = [i for i in range(3) if i != drop]
    P = [(v[keep[0]], v[keep[1]]) for v in (p, q, a, b, c)]
    p2, q2, a2, b2, c2 = P

    def o2(u, v, w):
        d = (v[0] - u[0]) * (w[1] - u[1]) - (v[1] - u[1]) * (w[0] - u[0])
        return (d > 0) - (d < 0)

    def in_tri(u):
        s = [o2(a2, b2, u), o2(b2, c2, u), o2(c2, a2, u)]
        nz = [v for v in s if v != 0]
        return all(v == nz[0] for v in nz)

    def seg_seg(u1, u2, v1, v2):
        d1, d2 = o2(u1, u2, v1), o2(u1, u2, v2)
        d3, d4 = o2(v1, v2, u1), o2(v1, v2, u2)
        if d1 * d2 < 0 and d3 * d4 < 0:
            return True

        def on(u, v, w):
            return o2(u, v, w) == 0 and min(u[0], v[0]) <= w[0] <= max(u[0], v[0]) and \
                min(u[1], v[1]) <= w[1] <= max(u[1], v[1])
        return on(u1, u2, v1) or on(u1, u2, v2) or on(v1, v2, u1) or on(v1, v2, u2)

    if in_tri(p2) or in_tri(q2):
        return True
    return any(seg_seg(p2, q2, e0, e1) for e0, e1 in ((a2, b2), (b2, c2), (c2, a2)))


def _cross(u, v):
    return [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]


def _sub(u, v):
    return [u[i] - v[i] for i in range(3)]


def _hull_segment(T):
    """Endpoints of a degenerate (collinear) triangle's extent."""
    best = (T[0], T[1])
    dmax = -1
    for i in range(3):
        for j in range(i + 1, 3):
            d = sum((T[i][k] - T[j][k]) ** 2 for k in range(3))
            if d > dmax:
                dmax, best = d, (T[i], T[j])
    return best


def _seg_seg(p, q, r, s) -> bool:
    """Closed 3-D segments pq and rs intersect (exact)."""
    if _orient(p, q, r, s) != 0:
        return False
    n = _cross(_sub(q, p), _sub(s, r))
    if all(v == 0 for v in n):
        n = _cross(_sub(q, p), _sub(r, p))
    if all(v == 0 for v in n):
        # all collinear: overlap of 1-D intervals along the dominant direction
        d = _sub(q, p) if any(_sub(q, p)) else _sub(s, r)
        ax = max(range(3), key=lambda i: abs(d[i]))
        a0, a1 = sorted((p[ax], q[ax]))
        b0, b1 = sorted((r[ax], s[ax]))
        if not any(d):
            return p == r
        return max(a0, b0) <= min(a1, b1)
    drop = max(range(3), key=lambda i: abs(n[i]))
    keep = [i for i in range(3) if i != drop]
    P = [(v[keep[0]], v[keep[1]]) for v in (p, q, r, s)]

    def o2(u, v, w):
        d = (v[0] - u[0]) * (w[1] - u[1]) - (v[1] - u[1]) * (w[0] - u[0])
        return (d > 0) - (d < 0)

    def on(u, v, w):
        return o2(u, v, w) == 0 and min(u[0], v[0]) <= w[0] <= max(u[0], v[0]) and \
            min(u[1], v[1]) <= w[1] <= max(u[1], v[1])
    u1, u2, v1, v2 = P
    d1, d2, d3, d4 = o2(u1, u2, v1), o2(u1, u2, v2), o2(v1, v2, u1), o2(v1, v2, u2)
    if d1 * d2 < 0 and d3 * d4 < 0:
        return True
    return on(u1, u2, v1) or on(u1, u2, v2) or on(v1, v2, u1) or on(v1, v2, u2)


def _degenerate(T) -> bool:
    return all(v == 0 for v in _cross(_sub(T[1], T[0]), _sub(T[2], T[0])))


def tri_tri_exact(A, B) -> bool:
    A = [[_exact_int(v) for v in row] for row in A]
    B = [[_exact_int(v) for v in row] for row in B]
    for k in range(3):
        if max(r[k] for r in A) < min(r[k] for r in B) or max(r[k] for r in B) < min(r[k] for r in A):
            return False
    da, db = _degenerate(A), _degenerate(B)
    if da and db:
        return _seg_seg(*_hull_segment(A), *_hull_segment(B))
    if da:
        return _seg_tri(*_hull_segment(A), *B)
    if db:
        return _seg_tri(*_hull_segment(B), *A)
    for (p, q) in ((A[0], A[1]), (A[1], A[2]), (A[2], A[0])):
        if _seg_tri(p, q, B[0], B[1], B[2]):
            return True
    for (p, q) in ((B[0], B[1]), (B[1], B[2]), (B[2], B[0])):
        if _seg_tri(p, q, A[0], A[1], A[2]):
            return True
    return False


def count_tangles(x32: np.ndarray, tris: np.ndarray):
    """Number of intersecting pairs of vertex-disjoint triangles at the FP32
    positions x32 (exact decision)."""
    x32 = np.asarray(x32, np.float32)
    hits, und, n_und, first = native.tangles(x32, tris, cap=1 << 16)
    if n_und > len(und):
        raise RuntimeError("too many undecided pairs for the exact pass")
    extra = 0
    for t, u in und:
        if tri_tri_exact(x32[tris[t]], x32[tris[u]]):
            extra += 1
    return hits + extra
