"""Exact labels of grid points (eq. 2) in rational arithmetic on the input
doubles: the re-decision of the points the FP64 oracle leaves undecided.

TEST INFRASTRUCTURE ONLY (with the rest of oracle/): the tests, the smoke check
and the CPU-baseline leg of the benchmark use it, never the product path.

The label follows the same three cases as the FP64 oracle (the definition of
the SES through probe balls that overlap no atom, section 1, and eq. 2), with
every comparison made exactly.  With s_i = r_i + rho (an exact real sum of two
doubles):

  1. |x - c_i|^2 <= r_i^2 for some i                       -> 1 (inside)
  2. |x - c_i|^2 >= s_i^2 for every i (x lies in A)          -> 0
  3. otherwise 0 iff an admissible candidate lies strictly within rho of x:
     (V) a concave probe position p of the oracle's list (atoms i < j < k,
         side sigma): the exact point on the three SAS spheres,
     (F) the radial projection y_i of x onto S_i, within rho iff
         |x - c_i| < s_i + rho, admissible iff |y_i - c_k| >= s_k for every
         other atom k,
     (E) the nearest point q of the circle S_i ^ S_j, admissible iff
         |q - c_k| >= s_k for every other atom k.

Every quantity below is a rational function of the input doubles except for
square roots, and each comparison is brought to the sign of a + b sqrt(X)
with rational a, b, X (decided by squaring under sign analysis):

  (F) with D = |x - c_i|^2 and u = (x - c_i) / sqrt(D), |y - c_k|^2 - s_k^2 =
      s_i^2 + d_ik^2 - s_k^2 - 2 s_i u.(c_k - c_i); multiplied by sqrt(D) > 0
      this is N sqrt(D) - L with N = s_i^2 + d_ik^2 - s_k^2 and
      L = 2 s_i (x - c_i).(c_k - c_i).
  (E) v = c_j - c_i, D = |v|^2; the circle's centre o = c_i + alpha v with
      alpha = (s_i^2 - s_j^2 + D) / 2D and R^2 = s_i^2 - alpha^2 D are rational.
      With w = x - o, w_perp = w - (w.v / D) v and b^2 = |w_perp|^2,
      |x - q|^2 = |w|^2 + R^2 - 2 R b, so "within rho" is the sign of
      2 sqrt(R^2 b^2) - (|w|^2 + R^2 - rho^2).  For q = o + R w_perp / b,
      (|q - c_k|^2 - s_k^2) b / R = N_k sqrt(b^2 / R^2) + 2 M_k with
      N_k = |o - c_k|^2 + R^2 - s_k^2 and M_k = (o - c_k).w_perp.  On the axis
      (b = 0) every circle point is equally near; the candidate is then taken
      in a fixed direction perpendicular to v (whichever is taken, a crossed
      circle's admissible arc ends at probe positions that lie equally near,
      so the label does not depend on it).
  (V) a = c_j - c_i, b = c_k - c_i, m = a x b.  The point z on the line of the
      two radical planes (2 a.z = s_i^2 - s_j^2 + |a|^2, 2 b.z = s_i^2 - s_k^2
      + |b|^2) with m.z = 0 is z = (A (b x m) + B (m x a)) / (2 |m|^2), and
      p = c_i + z + sigma sqrt(T) m with T = (s_i^2 - |z|^2) / |m|^2 (sigma
      = +1 is the side where (p - c_i).m > 0, the side convention of the
      probe list).  With e = x - c_i - z, |x - p|^2 - rho^2 =
      |e|^2 + T |m|^2 - rho^2 - 2 sigma sqrt(T) m.e.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np


def _sgn(v) -> int:
    return (v > 0) - (v < 0)


def sign_sqrt_sum(a, b, X) -> int:
    """Sign of a + b sqrt(X) for rationals a, b and X >= 0."""
    if X == 0 or b == 0:
        return _sgn(a)
    sa, sb = _sgn(a), _sgn(b)
    if sa == 0:
        return sb
    if sa == sb:
        return sa
    return sa * _sgn(a * a - b * b * X)


def _dot(p, q):
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2]


def _sub(p, q):
    return (p[0] - q[0], p[1] - q[1], p[2] - q[2])


def _cross(p, q):
    return (p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0])


def _scale(p, s):
    return (p[0] * s, p[1] * s, p[2] * s)


def _add(p, q):
    return (p[0] + q[0], p[1] + q[1], p[2] + q[2])


class ExactLabeller:
    """Exact labels for one molecule.

    centres [n,3], radii [n] (float64), probe radius; the concave probe list as
    triples (ascending atom ids) and sides.  Atoms near a point are found in
    FP64 with a generous margin (a superset); every decision is exact."""

    def __init__(self, centres, radii, probe, vert_atoms, vert_sign, vert_pos=None):
        self.c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        self.r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        self.rho = float(probe)
        self.s64 = self.r + self.rho
        self.smax = float(self.s64.max())
        self.R = Fr(self.rho)
        self.va = np.asarray(vert_atoms, dtype=np.int64).reshape(-1, 3)
        self.vs = np.asarray(vert_sign, dtype=np.int64).reshape(-1)
        self.vp = None if vert_pos is None else np.asarray(vert_pos, dtype=np.float64).reshape(-1, 3)
        self._C = {}
        self._N = {}
        self._vexact = {}

    # exact inputs, converted on first use
    def C(self, i):
        v = self._C.get(i)
        if v is None:
            v = (tuple(Fr(float(t)) for t in self.c[i]), Fr(float(self.r[i])))
            self._C[i] = v
        return v

    def s(self, i):
        return self.C(i)[1] + self.R

    def nbrs(self, i):
        """Atoms k != i whose SAS balls overlap ball i (superset by 1e-6 A)."""
        v = self._N.get(i)
        if v is None:
            d = np.linalg.norm(self.c - self.c[i], axis=1)
            v = np.flatnonzero(d < self.s64 + self.s64[i] + 1e-6)
            v = [int(k) for k in v if k != i]
            self._N[i] = v
        return v

    def _vertex(self, q):
        """(c_i, z, m, |m|^2, T, sigma) of probe position q."""
        v = self._vexact.get(q)
        if v is None:
            i, j, k = (int(t) for t in self.va[q])
            ci, _ = self.C(i)
            cj, _ = self.C(j)
            ck, _ = self.C(k)
            si, sj, sk = self.s(i), self.s(j), self.s(k)
            a = _sub(cj, ci)
            b = _sub(ck, ci)
            m = _cross(a, b)
            mm = _dot(m, m)
            A = si * si - sj * sj + _dot(a, a)
            B = si * si - sk * sk + _dot(b, b)
            z = _scale(_add(_scale(_cross(b, m), A), _scale(_cross(m, a), B)), 1 / (2 * mm))
            T = (si * si - _dot(z, z)) / mm
            v = (ci, z, m, mm, T, int(self.vs[q]))
            self._vexact[q] = v
        return v

    def label(self, x) -> int:
        x64 = np.asarray(x, dtype=np.float64)
        X = tuple(Fr(float(t)) for t in x64)
        rho = self.R
        dist = np.linalg.norm(self.c - x64, axis=1)
        near = np.flatnonzero(dist < self.s64 + self.rho + 1e-6)
        D = {}
        inU = False
        for i in near:
            i = int(i)
            ci, ri = self.C(i)
            e = _sub(X, ci)
            Di = _dot(e, e)
            D[i] = Di
            if Di <= ri * ri:
                return 1
            si = ri + rho
            if Di < si * si:
                inU = True
        if not inU:
            return 0
        # (V) concave probe positions
        if len(self.va):
            if self.vp is not None:
                cand = np.flatnonzero(np.linalg.norm(self.vp - x64, axis=1) < self.rho + 1e-6)
            else:
                cand = range(len(self.va))
            for q in cand:
                ci, z, m, mm, T, sg = self._vertex(int(q))
                e = _sub(_sub(X, ci), z)
                P = _dot(e, e) + T * mm - rho * rho
                if sign_sqrt_sum(P, -2 * sg * _dot(m, e), T) < 0:
                    return 0
        # (F) radial projections
        for i, Di in D.items():
            si = self.s(i)
            if not (Di < (si + rho) ** 2):
                continue
            ci, _ = self.C(i)
            e = _sub(X, ci)
            ok = True
            for k in self.nbrs(i):
                ck, _ = self.C(k)
                sk = self.s(k)
                v = _sub(ck, ci)
                N = si * si + _dot(v, v) - sk * sk
                L = 2 * si * _dot(e, v)
                if sign_sqrt_sum(-L, N, Di) < 0:
                    ok = False
                    break
            if ok:
                return 0
        # (E) nearest circle points
        for i in D:
            for j in self.nbrs(i):
                if j <= i or j not in D:
                    continue
                if self._circle_candidate(X, i, j):
                    return 0
        return 1

    def _circle_candidate(self, X, i, j) -> bool:
        rho = self.R
        ci, _ = self.C(i)
        cj, _ = self.C(j)
        si, sj = self.s(i), self.s(j)
        v = _sub(cj, ci)
        Dv = _dot(v, v)
        if not ((si - sj) ** 2 < Dv < (si + sj) ** 2):
            return False  # the spheres meet in no circle
        alpha = (si * si - sj * sj + Dv) / (2 * Dv)
        o = _add(ci, _scale(v, alpha))
        R2 = si * si - alpha * alpha * Dv
        w = _sub(X, o)
        ww = _dot(w, w)
        wp = _sub(w, _scale(v, _dot(w, v) / Dv))
        b2 = _dot(wp, wp)
        P = ww + R2 - rho * rho
        if not (sign_sqrt_sum(-P, 2, R2 * b2) > 0):
            return False
        if b2 == 0:
            # on the axis: a fixed perpendicular direction
            ax = int(np.argmin(np.abs([float(t) for t in v])))
            e = tuple(Fr(1) if t == ax else Fr(0) for t in range(3))
            wp = _sub(e, _scale(v, _dot(e, v) / Dv))
            b2 = _dot(wp, wp)
        W = b2 / R2
        for k in self.nbrs(i):
            if k == j:
                continue
            ck, _ = self.C(k)
            sk = self.s(k)
            oc = _sub(o, ck)
            Nk = _dot(oc, oc) + R2 - sk * sk
            Mk = _dot(oc, wp)
            if sign_sqrt_sum(2 * Mk, Nk, W) < 0:
                return False
        return True


def exact_labels(centres, radii, probe, vert_atoms, vert_sign, points, vert_pos=None):
    """Exact labels (uint8) of points [m,3]."""
    E = ExactLabeller(centres, radii, probe, vert_atoms, vert_sign, vert_pos)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return np.array([E.label(p) for p in pts], dtype=np.uint8)
