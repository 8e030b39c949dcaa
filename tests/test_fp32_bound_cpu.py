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
