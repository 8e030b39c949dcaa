"""Marching-cubes mesh, area and volume from labels and crossing records.

TEST INFRASTRUCTURE ONLY (with the rest of oracle/).

Section 2.2 of the paper turns the Eulerian output into a triangle mesh by
marching cubes, and its appendix table reports each complex's surface area and
volume.  The mesh here: each cube of eight axis-adjacent grid points with mixed
labels is cut by triangles whose corners are the crossing points of its edges
(p = s + (1 - lambda) h e, eq. 4).  The cases follow one rule: on each face
the crossing points are joined in pairs -- where all four edges of a face cross
(the inside corners diagonal), each inside corner is cut off -- the joins of
the six faces close into loops, each loop is oriented with its normal from the
inside ends of its edges to their outside ends, started at its smallest edge
and cut into a fan of triangles.  Edge numbering: edge 4a + r runs along axis
a from the cube corner whose other two coordinates are the bits of r (lower bit
first, in axis order); corner c = x + 2y + 4z.
"""
from __future__ import annotations

import numpy as np


def _corner(c):
    return np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])


def _edge_ends(e):
    a, r = divmod(e, 4)
    lo = [0, 0, 0]
    others = [b for b in range(3) if b != a]
    lo[others[0]] = r & 1
    lo[others[1]] = (r >> 1) & 1
    hi = list(lo)
    hi[a] = 1
    return lo[0] + 2 * lo[1] + 4 * lo[2], hi[0] + 2 * hi[1] + 4 * hi[2]


def _edge_between(c0, c1):
    p, q = _corner(c0), _corner(c1)
    a = int(np.flatnonzero(p != q)[0])
    others = [b for b in range(3) if b != a]
    return 4 * a + int(p[others[0]]) + 2 * int(p[others[1]])


def case_table():
    """{configuration: [(e0, e1, e2), ...]} for the 256 corner configurations."""
    table = {}
    for cfg in range(256):
        inside = [(cfg >> c) & 1 for c in range(8)]
        links = {}
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            for side in (0, 1):
                ring = []
                for u, v in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    xyz = [0, 0, 0]
                    xyz[a], xyz[b], xyz[c] = side, u, v
                    ring.append(xyz[0] + 2 * xyz[1] + 4 * xyz[2])
                cut = [q for q in range(4) if inside[ring[q]] != inside[ring[(q + 1) % 4]]]
                pairs = []
                if len(cut) == 2:
                    pairs.append((_edge_between(ring[cut[0]], ring[(cut[0] + 1) % 4]),
                                  _edge_between(ring[cut[1]], ring[(cut[1] + 1) % 4])))
                elif len(cut) == 4:
                    for q in range(4):
                        if inside[ring[q]]:
                            pairs.append((_edge_between(ring[(q + 3) % 4], ring[q]),
                                          _edge_between(ring[q], ring[(q + 1) % 4])))
                for x, y in pairs:
                    links.setdefault(x, []).append(y)
                    links.setdefault(y, []).append(x)
        tris = []
        done = set()
        for start in sorted(links):
            if start in done:
                continue
            loop = [start]
            done.add(start)
            prev, cur = None, start
            while True:
                nxt = [v for v in links[cur] if v != prev and v not in done]
                if not nxt:
                    break
                prev, cur = cur, nxt[0]
                loop.append(cur)
                done.add(cur)
            mids, D = [], np.zeros(3)
            for e in loop:
                c0, c1 = _edge_ends(e)
                p0, p1 = _corner(c0), _corner(c1)
                mids.append(0.5 * (p0 + p1))
                D += (p1 - p0) if inside[c0] else (p0 - p1)
            N = np.zeros(3)
            for q in range(len(loop)):
                u, v = mids[q], mids[(q + 1) % len(loop)]
                N += np.cross(u, v)
            if N @ D < 0:
                loop = loop[::-1]
            s = loop.index(min(loop))
            loop = loop[s:] + loop[:s]
            tris += [(loop[0], loop[q], loop[q + 1]) for q in range(1, len(loop) - 1)]
        table[cfg] = tris
    return table


_TABLE = None


def mesh(labels, lo, h, keys, lam):
    """Triangles of the mesh as record-index triples [m, 3] (in cube order,
    each cube's in table order) and the vertices (one per record, relative to
    the grid origin) [n, 3]."""
    global _TABLE
    if _TABLE is None:
        _TABLE = case_table()
    L = np.asarray(labels, dtype=np.uint8)
    nz, ny, nx = L.shape
    keys = np.asarray(keys, dtype=np.int64)
    lam = np.asarray(lam, dtype=np.float64)
    idx = keys // 3
    axis = keys % 3
    ijk = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1)
    verts = np.stack([(float(lo[a]) + ijk[:, a].astype(np.float64) * float(h)) - float(lo[a])
                      for a in range(3)], axis=1)
    verts[np.arange(len(keys)), axis] += (1.0 - lam) * h
    cfg = np.zeros((nz - 1, ny - 1, nx - 1), dtype=np.int64)
    for c in range(8):
        x, y, z = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cfg |= L[z:nz - 1 + z, y:ny - 1 + y, x:nx - 1 + x].astype(np.int64) << c
    kk, jj, ii = np.nonzero((cfg != 0) & (cfg != 255))
    order = np.lexsort((ii, jj, kk))
    kk, jj, ii = kk[order], jj[order], ii[order]
    cf = cfg[kk, jj, ii]
    out = []
    for k, j, i, c in zip(kk, jj, ii, cf):
        for tri in _TABLE[int(c)]:
            row = []
            for e in tri:
                a, r = divmod(e, 4)
                off = [0, 0, 0]
                others = [b for b in range(3) if b != a]
                off[others[0]] = r & 1
                off[others[1]] = (r >> 1) & 1
                g = (i + off[0]) + nx * ((j + off[1]) + ny * (k + off[2]))
                row.append(3 * g + a)
            out.append(row)
    tkeys = np.array(out, dtype=np.int64).reshape(-1, 3)
    tri = np.searchsorted(keys, tkeys)
    tri = np.minimum(tri, max(len(keys) - 1, 0))
    assert len(keys) == 0 or np.all(keys[tri] == tkeys), "a cut edge has no crossing record"
    return tri.astype(np.int64), verts


def area_volume(tri, verts):
    """Sum of triangle areas; enclosed volume by the divergence theorem."""
    v0, v1, v2 = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", v0, np.cross(v1, v2)).sum() / 6.0
    return float(area), float(vol)


def closed_and_oriented(tri):
    """Every mesh edge is used by exactly two triangles, in opposite directions."""
    d = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    fwd = {}
    for a, b in map(tuple, d):
        fwd[(a, b)] = fwd.get((a, b), 0) + 1
    return all(n == 1 and fwd.get((b, a), 0) == 1 for (a, b), n in fwd.items())
