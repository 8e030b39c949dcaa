"""Comparison of the HIP path's outputs with the oracle's (test helper)."""
import numpy as np

POS_TOL = 1e-6      # angstrom, intersection positions
NORMAL_TOL = 1e-6   # per component, unit normals


def compare_vertices(gpu_vertices, oracle):
    p, a, s = gpu_vertices
    po, ao, so = oracle.vertices()
    kg = {(int(x[0]), int(x[1]), int(x[2]), int(sg)): q for q, x, sg in zip(p, a, s)}
    ko = {(int(x[0]), int(x[1]), int(x[2]), int(sg)): q for q, x, sg in zip(po, ao, so)}
    assert len(kg) == len(p), "duplicate concave probe positions from the HIP path"
    assert set(kg) == set(ko), (len(set(kg) - set(ko)), len(set(ko) - set(kg)))
    if ko:
        # the two constructions (circle-sphere angle against trilateration)
        # agree to within 2e-15 of the coordinates' size on every workload
        # measured (at most 1.4e-13 A at 69 A); 2e-14 of it, about 180 units
        # in the last place, leaves a tenfold margin
        err = max(np.max(np.abs(kg[k] - ko[k])) for k in ko)
        tol = 2e-14 * max(1.0, float(np.max(np.abs(po))))
        assert err < tol, (err, tol)
    return len(ko)


def compare_labels(gpu_labels, oracle_labels):
    assert gpu_labels.shape == oracle_labels.shape
    diff = np.flatnonzero(gpu_labels.reshape(-1) != oracle_labels.reshape(-1))
    assert diff.size == 0, f"{diff.size} labels differ, first at flat index {diff[:5]}"


def crossing_points(res, lo, h, dims):
    """The crossing position of every record (key = 3 * point + axis; the
    crossing is at lambda * s + (1 - lambda) * (s + h e_axis))."""
    key = res["key"]
    nx, ny, _ = dims
    axis = key % 3
    idx = key // 3
    p = np.stack([lo[0] + (idx % nx) * h, lo[1] + ((idx // nx) % ny) * h,
                  lo[2] + (idx // (nx * ny)) * h], axis=1)
    p[np.arange(len(key)), axis] += (1 - res["lam"]) * h
    return p


def surface_residual(oracle, ptype, atoms, x):
    """| distance from x to the claimed patch's whole surface - its radius |:
    the atom's sphere (type 1), the torus swept by the probe around the pair's
    circle (type 2), the nearer probe sphere of the triple (type 3).  Also
    returns the probe centre used for type 3 (nan elsewhere)."""
    c, r, rho = oracle.c, oracle.r, oracle.probe
    s = r + rho
    out = np.full(len(x), np.inf)
    probe = np.full((len(x), 3), np.nan)
    t1 = ptype == 1
    out[t1] = np.abs(np.linalg.norm(x[t1] - c[atoms[t1, 0]], axis=1) - r[atoms[t1, 0]])
    t2 = np.flatnonzero(ptype == 2)
    if t2.size:
        a, b = atoms[t2, 0], atoms[t2, 1]
        v = c[b] - c[a]
        d = np.linalg.norm(v, axis=1)
        n = v / d[:, None]
        t = (s[a] ** 2 - s[b] ** 2 + d ** 2) / (2 * d)
        R = np.sqrt(np.maximum(s[a] ** 2 - t ** 2, 0.0))
        w = x[t2] - (c[a] + t[:, None] * n)
        along = np.sum(w * n, axis=1)
        perp = np.linalg.norm(w - along[:, None] * n, axis=1)
        out[t2] = np.abs(np.hypot(perp - R, along) - rho)
    t3 = np.flatnonzero(ptype == 3)
    if t3.size:
        pv, av, _ = oracle.vertices()
        by = {}
        for q, tr in enumerate(av):
            by.setdefault(tuple(int(v) for v in tr), []).append(pv[q])
        for m in t3:
            best = np.inf
            for pp in by.get(tuple(int(v) for v in atoms[m]), []):
                e = abs(np.linalg.norm(x[m] - pp) - rho)
                if e < best:
                    best, probe[m] = e, pp
            out[m] = best
    return out, probe


def cusp_mask(res, centres, lo, h, dims, tol=1e-6):
    """Saddle crossings on (or within tol of) the axis through their two atoms:
    there every circle point is equally near, so the normal is not unique."""
    key = res["key"]
    nx, ny, _ = dims
    axis = key % 3
    idx = key // 3
    p = np.stack([lo[0] + (idx % nx) * h, lo[1] + ((idx // nx) % ny) * h,
                  lo[2] + (idx // (nx * ny)) * h], axis=1)
    p[np.arange(len(key)), axis] += (1 - res["lam"]) * h
    sad = res["patch_type"] == 2
    out = np.zeros(len(key), bool)
    if sad.any():
        a = centres[res["atoms"][sad, 0]]
        b = centres[res["atoms"][sad, 1]]
        n = (b - a) / np.linalg.norm(b - a, axis=1, keepdims=True)
        w = p[sad] - a
        perp = w - np.sum(w * n, axis=1, keepdims=True) * n
        out[sad] = np.linalg.norm(perp, axis=1) < tol
    return out


TIE_RESID = 1e-10   # angstrom: a crossing on two surfaces at once (owner tie)
GEN_RESID = 1e-9    # angstrom: a normal consistent with the surface it names


def generator_residual(oracle, ptype, atoms, x, n):
    """How far the normal n at x is from the normal of the claimed surface: the
    point x - r n must be the atom's centre (convex), x + rho n a point of the
    pair's circle (saddle) or one of the triple's probe positions (concave)."""
    c, r, rho = oracle.c, oracle.r, oracle.probe
    s = r + rho
    out = np.full(len(x), np.inf)
    t1 = ptype == 1
    out[t1] = np.linalg.norm(x[t1] - r[atoms[t1, 0], None] * n[t1] - c[atoms[t1, 0]], axis=1)
    t2 = np.flatnonzero(ptype == 2)
    if t2.size:
        a, b = atoms[t2, 0], atoms[t2, 1]
        v = c[b] - c[a]
        d = np.linalg.norm(v, axis=1)
        ax = v / d[:, None]
        t = (s[a] ** 2 - s[b] ** 2 + d ** 2) / (2 * d)
        R = np.sqrt(np.maximum(s[a] ** 2 - t ** 2, 0.0))
        q = x[t2] + rho * n[t2] - (c[a] + t[:, None] * ax)
        along = np.sum(q * ax, axis=1)
        out[t2] = np.hypot(np.linalg.norm(q - along[:, None] * ax, axis=1) - R, along)
    t3 = np.flatnonzero(ptype == 3)
    if t3.size:
        pv, av, _ = oracle.vertices()
        by = {}
        for q, tr in enumerate(av):
            by.setdefault(tuple(int(v) for v in tr), []).append(pv[q])
        for m in t3:
            p = x[m] + rho * n[m]
            out[m] = min((np.linalg.norm(p - pp) for pp in by.get(tuple(int(v) for v in atoms[m]),
                                                                    [])), default=np.inf)
    return out


def compare_edges(res, oracle, lo, h, dims, ref_labels=None, log=True):
    """Edge set identical to the oracle's crossing set; lambda (as a position
    along the edge) within POS_TOL; patch tags equal and normals within
    NORMAL_TOL -- except at owner ties.

    A record whose owner or normal differs from the oracle's is an owner tie,
    accepted only where both claimed surfaces pass through the crossing point
    (to TIE_RESID: two patches meet there, or one probe sphere is reported by
    several triples) and each side's normal is the normal of the surface it
    names (to GEN_RESID); their normals may then differ by the crease between
    the patches.  Normals at saddle cusps (crossings on the axis of a spindle
    torus) are not unique and are not compared.  Returns (records, owner
    ties); the tie count is printed."""
    from oracle.oracle import crossing_keys
    key = res["key"]
    assert np.all(np.diff(key) > 0), "keys not strictly ascending"
    if ref_labels is not None:
        want = crossing_keys(ref_labels)
        assert np.array_equal(key, want), (len(key), len(want))
    rec = oracle.edges(lo, h, dims, key)
    assert np.all(rec["status"] == 1)
    assert set(np.unique(res["patch_type"])) <= {1, 2, 3}
    assert np.all(np.abs(np.linalg.norm(res["normal"], axis=1) - 1) < 1e-12)
    dpos = np.abs(rec["lam"] - res["lam"]) * h
    assert dpos.max(initial=0.0) < POS_TOL, dpos.max()
    dn = np.abs(rec["normal"] - res["normal"]).max(axis=1) if len(key) else np.zeros(0)
    tag_same = (rec["type"] == res["patch_type"]) & np.all(rec["atoms"] == res["atoms"], axis=1)
    cusp = cusp_mask(res, oracle.c, lo, h, dims)
    tie = (~tag_same | (dn >= NORMAL_TOL)) & ~cusp
    diff = np.flatnonzero(tie)
    creases = 0
    if diff.size:
        x = crossing_points(res, lo, h, dims)[diff]
        resid, _ = surface_residual(oracle, res["patch_type"][diff], res["atoms"][diff], x)
        resid_o, _ = surface_residual(oracle, rec["type"][diff], rec["atoms"][diff], x)
        assert resid.max() < TIE_RESID, ("HIP owner off the crossing", resid.max())
        assert resid_o.max() < TIE_RESID, ("owners differ away from a tie", resid_o.max())
        g = generator_residual(oracle, res["patch_type"][diff], res["atoms"][diff], x,
                               res["normal"][diff])
        g_o = generator_residual(oracle, rec["type"][diff], rec["atoms"][diff], x,
                                 rec["normal"][diff])
        assert g.max() < GEN_RESID, ("HIP normal is not its surface's", g.max())
        assert g_o.max() < GEN_RESID, ("oracle normal is not its surface's", g_o.max())
        creases = int((dn[diff] >= NORMAL_TOL).sum())
    if log:
        print(f"edges: {len(key)} records, {diff.size} owner ties ({creases} at creases)",
              flush=True)
    return len(key), int(diff.size)
