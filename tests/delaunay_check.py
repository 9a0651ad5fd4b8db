"""Validity of linear interpolation where the Delaunay triangulation is not
unique (exactly cocircular points, Algorithm 1 on lattice inputs).

Several triangulations are then correct, and a texel on a shared circle may
take its value from any of them.  The check accepts a texel's linear height
when it equals barycentric interpolation in some triangle that contains the
texel and whose open circumcircle holds no input point, i.e. a triangle of
some Delaunay triangulation.  Candidates: the triangle SciPy's Delaunay
returns for the texel (its circle is empty) and every other triangle whose
vertices lie exactly on that circle (exact integer in-circle tests).
Texels outside the convex hull must carry the nearest-neighbour value.
"""
import itertools

import numpy as np
from scipy.spatial import Delaunay


def _orient(a, b, c):
    return (int(b[0]) - int(a[0])) * (int(c[1]) - int(a[1])) - (int(b[1]) - int(a[1])) * (int(c[0]) - int(a[0]))


def _incircle(a, b, c, d):
    rows = []
    for p in (a, b, c):
        dx, dy = int(p[0]) - int(d[0]), int(p[1]) - int(d[1])
        rows.append((dx, dy, dx * dx + dy * dy))
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0)


def _on_circle(P, tri):
    """Indices of all points exactly on the circumcircle of CCW tri; asserts
    none is strictly inside."""
    a, b, c = (P[i] for i in tri)
    d = P.astype(np.float64) - a
    ab, ac = (b - a).astype(np.float64), (c - a).astype(np.float64)
    la, lb, lc = 0.0, ab @ ab, ac @ ac
    # in-circle determinant with a as the origin (float filter; the 3x3
    # determinant of rows b - a, c - a, d - a is minus the in-circle value)
    dd = (d ** 2).sum(1)
    det = -(ab[0] * (ac[1] * dd - lc * d[:, 1]) - ab[1] * (ac[0] * dd - lc * d[:, 0])
            + lb * (ac[0] * d[:, 1] - ac[1] * d[:, 0]))
    near = np.nonzero(np.abs(det) <= 1e9)[0]
    out = []
    for i in near:
        s = _incircle(a, b, c, P[i])
        assert s <= 0, "SciPy triangle with a point strictly inside its circumcircle"
        if s == 0:
            out.append(int(i))
    # a clearly positive float value is strictly inside
    assert not np.any(det > 1e9), "SciPy triangle with a point strictly inside its circumcircle"
    return out


def check_linear_valid(P, zm, qx, qy, h_lin, h_nn, tol):
    """P [m, 2] int64 unique points, zm [m] heights (m), texel centres qx, qy
    (int arrays), h_lin / h_nn maps.  Returns (texels checked, texels where
    more than one value was admissible)."""
    P = np.asarray(P, np.int64)
    dt = Delaunay(P.astype(np.float64))
    Q = np.stack([np.ravel(qx), np.ravel(qy)], 1)
    s = dt.find_simplex(Q.astype(np.float64))
    hl, hn = np.ravel(h_lin), np.ravel(h_nn)
    cache = {}
    ambiguous = 0
    for t in range(len(Q)):
        q = Q[t]
        if s[t] < 0:
            # outside scipy's hull or on its boundary: either NN, or inside a
            # hull triangle touching q (boundary texels)
            tri = None
            for k, simp in enumerate(dt.simplices):
                a, b, c = (P[i] for i in simp)
                o = _orient(a, b, c)
                sg = 1 if o > 0 else -1
                if all(sg * _orient(*e, q) >= 0 for e in ((a, b), (b, c), (c, a))):
                    tri = k
                    break
            if tri is None:
                assert abs(hl[t] - hn[t]) <= tol, (t, hl[t], hn[t])
                continue
            s[t] = tri
        simp = tuple(int(i) for i in dt.simplices[s[t]])
        if simp not in cache:
            a, b, c = simp
            if _orient(P[a], P[b], P[c]) < 0:
                a, b = b, a
            cache[simp] = _on_circle(P, (a, b, c))
        circ = cache[simp]
        vals = []
        for a, b, c in itertools.combinations(circ, 3):
            o = _orient(P[a], P[b], P[c])
            if o == 0:
                continue
            if o < 0:
                a, b = b, a
                o = -o
            la, lb, lc = _orient(P[b], P[c], q), _orient(P[c], P[a], q), _orient(P[a], P[b], q)
            if la < 0 or lb < 0 or lc < 0:
                continue
            vals.append((la * zm[a] + lb * zm[b] + lc * zm[c]) / o)
        assert vals, t
        if max(vals) - min(vals) > tol:
            ambiguous += 1
        assert min(abs(v - hl[t]) for v in vals) <= tol, (t, hl[t], vals)
    return len(Q), ambiguous


def lattice_points(rng, spacing=2000, keep=0.6, H=48000):
    """Points on a square lattice of the window (many exactly cocircular
    squares), each kept with probability `keep`, with random heights."""
    k = np.arange(-H, H, spacing)
    U, V = np.meshgrid(k, k)
    sel = rng.random(U.size) < keep
    u, v = U.ravel()[sel], V.ravel()[sel]
    z = rng.integers(-5000, 5000, len(u))
    return u.astype(np.int64), v.astype(np.int64), z.astype(np.int64)
