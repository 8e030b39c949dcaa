"""The certified FP32 distance test of the classification (the FP32 path whose
uncertain decisions are re-taken in FP64): emulated here in float32 exactly as
the kernel evaluates it (FP64 offsets from the tile origin rounded to FP32, an
FP32 difference, an FP32 sum of squares with or without fused multiply-adds),
every decision the FP32 interval certifies must agree with the exact comparison
of |x - c|^2 with the threshold, also for distances placed within the bound of
the threshold.  The
bound: E = 4.01 u lam per component, c0 = 3 E (4 lam + E), thresholds
(t (1 -+ 2^-52) -+ c0)(1 -+ 4u) rounded outward to FP32."""
from fractions import Fraction

import numpy as np

U = 2.0 ** -24


def outward(x, up):
    f = np.float32(x)
    if up and float(f) < x:
        f = np.nextafter(f, np.float32(np.inf))
    if not up and float(f) > x:
        f = np.nextafter(f, np.float32(-np.inf))
    return f


def thresholds(t, lam):
    E = 4.01 * U * lam
    c0 = 3.0 * E * (4.0 * lam + E) + 1e-30
    lo = outward((t * (1.0 - 2.0 ** -52) - c0) * (1.0 - 4.0 * U), False)
    hi = outward((t * (1.0 + 2.0 ** -52) + c0) * (1.0 + 4.0 * U), True)
    return lo, hi


def fma32(a, b, c):
    # a * b is exact in float64 for float32 a, b; the sum is rounded once to
    # float64 and then to float32 (a double rounding that can only move the
    # result by one float32 ulp, far inside the 4u margin)
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def check(px, c, r, org, lam):
    fx = [np.float32(px[a] - org[a]) for a in range(3)]
    fc = [np.float32(c[a] - org[a]) for a in range(3)]
    d = [np.float32(fx[a] - fc[a]) for a in range(3)]
    s_plain = np.float32(np.float32(d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
    s_fma = fma32(d[2], d[2], fma32(d[1], d[1], np.float32(d[0] * d[0])))
    e2 = sum((Fraction(px[a]) - Fraction(c[a])) ** 2 for a in range(3))
    t = Fraction(r) * Fraction(r)
    lo, hi = thresholds(float(r) * float(r), lam)
    certain = 0
    for s in (s_plain, s_fma):
        if s < lo:
            assert e2 < t, (px, c, r)
            certain += 1
        elif s > hi:
            assert e2 > t, (px, c, r)
            certain += 1
    return certain


def test_certified_fp32_decisions_are_exact():
    rng = np.random.default_rng(12)
    h, T, smax = 0.25, 8, 3.2
    lam = (T - 1) * h + smax + 1e-3
    n_cert = n_tot = 0
    for q in range(4000):
        org = rng.uniform(-60.0, 60.0, 3)
        k = rng.integers(0, T, 3)
        px = org + k * h
        r = float(rng.choice([1.2, 1.52, 1.55, 1.7, 1.8]) + (0.0 if q % 2 else 1.4))
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        near = q % 4 < 2
        if near:
            # |x - c|^2 within a few FP32 rounding errors of the threshold:
            # decisions a too small bound would wrongly certify
            dist = np.sqrt(r * r + rng.uniform(-1.0, 1.0) * U * lam * r)
        else:
            dist = rng.uniform(0.0, 2.0 * r)
        c = px + dist * u
        if np.any(np.abs(c - org) > lam):
            continue
        k = check(px, c, r, org, lam)
        if not near:
            n_cert += k
            n_tot += 2
    assert n_tot > 2000
    # the bound is tight enough that most random decisions are certified
    assert n_cert > 0.6 * n_tot


def test_certified_fp32_decisions_1e8_samples():
    """The same check vectorised over 10^8 random (point, atom) pairs, half of
    them near the threshold at every scale up to three times the bound's
    absolute term.  The exact
    comparison is taken in float64 where its margin exceeds float64's own
    rounding (|e - t| > 1e-13 t, e and t each within a few ulps), else in
    rational arithmetic."""
    rng = np.random.default_rng(20250)
    h, T, smax = 0.25, 8, 3.2
    lam = (T - 1) * h + smax + 1e-3
    radii = np.array([1.2, 1.52, 1.55, 1.7, 1.8, 2.6, 2.92, 2.95, 3.1, 3.2])
    thr = {float(r): thresholds(float(r) * float(r), lam) for r in radii}
    E = 4.01 * U * lam
    c0 = 3.0 * E * (4.0 * lam + E)
    n_total = n_cert = n_exact = n_far = 0
    chunk = 5_000_000
    for _ in range(20):
        # grid coordinates as the kernel forms them, fl(lo + fl(i h)), for the
        # point and for its tile's origin: both offsets round to FP32
        lo = rng.uniform(-60.0, 60.0, (chunk, 3))
        ti = rng.integers(0, 64, (chunk, 3)) * T
        org = lo + ti * h
        px = lo + (ti + rng.integers(0, T, (chunk, 3))) * h
        ri = rng.integers(0, len(radii), chunk)
        r = radii[ri]
        u = rng.normal(size=(chunk, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        # half the pairs with |x - c|^2 - r^2 of either sign and log-uniform
        # size between 1e-5 and 3 times the bound's absolute term c0, so that
        # every scale of the FP32 error (about 4e-7 r^2 at most here) is
        # sampled: certified there only beyond the bound (thresholds without
        # their margins fail this test; the absolute term c0 covers the worst
        # case of the offsets' rounding, which random pairs do not reach)
        near = rng.random(chunk) < 0.5
        delta = rng.choice([-1.0, 1.0], chunk) * 3.0 * c0 * 10.0 ** rng.uniform(-5.0, 0.0, chunk)
        dist = np.where(near, np.sqrt(r * r + delta), rng.uniform(0.0, 2.0 * r))
        c = px + dist[:, None] * u
        keep = np.all(np.abs(c - org) <= lam, axis=1)
        px, c, org, r, ri = px[keep], c[keep], org[keep], r[keep], ri[keep]
        fx = (px - org).astype(np.float32)
        fc = (c - org).astype(np.float32)
        d = fx - fc  # float32
        s_plain = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        d64 = d.astype(np.float64)
        s_fma = (d64[:, 0] * d64[:, 0]).astype(np.float32)
        s_fma = (d64[:, 1] * d64[:, 1] + s_fma.astype(np.float64)).astype(np.float32)
        s_fma = (d64[:, 2] * d64[:, 2] + s_fma.astype(np.float64)).astype(np.float32)
        lo = np.array([thr[float(x)][0] for x in radii], dtype=np.float32)[ri]
        hi = np.array([thr[float(x)][1] for x in radii], dtype=np.float32)[ri]
        e64 = np.sum((px - c) ** 2, axis=1)
        t64 = r * r
        below = e64 < t64 * (1.0 - 1e-13)
        above = e64 > t64 * (1.0 + 1e-13)
        for s in (s_plain, s_fma):
            cert_lo, cert_hi = s < lo, s > hi
            # decisions the float64 comparison settles
            assert not np.any(cert_lo & above), "FP32 certified inside, exactly outside"
            assert not np.any(cert_hi & below), "FP32 certified outside, exactly inside"
            # the rest of the certified ones, exactly
            for q in np.flatnonzero((cert_lo | cert_hi) & ~below & ~above):
                e2 = sum((Fraction(px[q, a]) - Fraction(c[q, a])) ** 2 for a in range(3))
                t = Fraction(float(r[q])) ** 2
                assert (e2 < t) if cert_lo[q] else (e2 > t), q
                n_exact += 1
            n_cert += int(np.count_nonzero((cert_lo | cert_hi) & ~near[keep]))
        n_total += len(r)
        n_far += int(np.count_nonzero(~near[keep]))
    assert n_total >= 10 ** 8 * 0.9
    # the bound is tight enough that most random decisions are certified
    assert n_cert > 0.6 * 2 * n_far
