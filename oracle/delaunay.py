"""Hexatic order parameter with Delaunay neighbours, and its autocorrelation
time -- TEST INFRASTRUCTURE ONLY (oracle).

Only the tests may import this module; the HIP library and its binding never
call it, and it shares no code with them.

eq. (Psi), Sec. 2: Psi = N^-1 sum_k Psi_k with Psi_k = n_k^-1 sum_l
exp(6 i phi_kl) over the n_k Delaunay neighbours l of disk k; phi_kl is the
angle of the vector from k to l against the x axis.  The periodic box is
triangulated together with the periodic images of the disks near its edges;
scipy's Delaunay (Qhull) is the triangulation step, pinned in the tests by
the empty-circumcircle definition on small point sets.

eq. (tau), Sec. 2: C(dt) = <Psi*(t) Psi(t + dt)> / <Psi*(t) Psi(t)> over a
time series of Psi (the phase of Psi is arbitrary, so <Psi> = 0 is taken as
given and no mean is subtracted), and tau is the decay time of
C(dt) ~ exp(-dt / tau).
"""
import numpy as np


def _with_images(x, y, Lx, Ly, margin):
    """Points plus their periodic images within `margin` outside the box;
    returns (points [M, 2], original index of every point [M])."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    pts = [np.stack([x, y], axis=1)]
    ids = [np.arange(n)]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            if sx == 0 and sy == 0:
                continue
            px, py = x + sx * Lx, y + sy * Ly
            keep = (px > -margin) & (px < Lx + margin) & (py > -margin) & (py < Ly + margin)
            pts.append(np.stack([px[keep], py[keep]], axis=1))
            ids.append(np.nonzero(keep)[0])
    return np.concatenate(pts), np.concatenate(ids)


def delaunay_neighbours(x, y, Lx, Ly, margin=None):
    """Delaunay neighbours of every disk of a periodic Lx x Ly box.

    Returns (offsets, ids): per disk k an array [n_k, 2] of vectors from k to
    the neighbour images, and an array [n_k] of the neighbours' indices."""
    from scipy.spatial import Delaunay
    n = len(x)
    if margin is None:
        spacing = np.sqrt(Lx * Ly / n)
        margin = min(0.5 * min(Lx, Ly), 8.0 * spacing)
    pts, orig = _with_images(x, y, Lx, Ly, margin)
    tri = Delaunay(pts)
    # every triangle at a disk of the box must have its circumcircle inside
    # the imaged region: then no missing image can lie in it, and the
    # triangles at the box's disks are those of the periodic point set
    s = tri.simplices[np.any(tri.simplices < n, axis=1)]
    a, b, c = pts[s[:, 0]], pts[s[:, 1]], pts[s[:, 2]]
    d = 2.0 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
    aa, bb, cc = (a * a).sum(1), (b * b).sum(1), (c * c).sum(1)
    ux = (aa * (b[:, 1] - c[:, 1]) + bb * (c[:, 1] - a[:, 1]) + cc * (a[:, 1] - b[:, 1])) / d
    uy = (aa * (c[:, 0] - b[:, 0]) + bb * (a[:, 0] - c[:, 0]) + cc * (b[:, 0] - a[:, 0])) / d
    r = np.sqrt((a[:, 0] - ux) ** 2 + (a[:, 1] - uy) ** 2)
    if (np.any(ux - r < -margin) or np.any(ux + r > Lx + margin) or np.any(uy - r < -margin)
            or np.any(uy + r > Ly + margin)):
        raise ValueError("image margin too small for the Delaunay triangles at the box's disks")
    indptr, indices = tri.vertex_neighbor_vertices
    offsets, ids = [], []
    for k in range(n):
        nb = indices[indptr[k]:indptr[k + 1]]
        offsets.append(pts[nb] - pts[k])
        ids.append(orig[nb])
    return offsets, ids


def psi6_delaunay(x, y, Lx, Ly, margin=None):
    """(Psi, per-disk Psi_k [N] complex, neighbour counts [N]) per eq. (Psi)."""
    offsets, _ = delaunay_neighbours(x, y, Lx, Ly, margin)
    n = len(offsets)
    psi_k = np.zeros(n, dtype=np.complex128)
    counts = np.zeros(n, dtype=np.int64)
    for k, v in enumerate(offsets):
        counts[k] = len(v)
        if len(v):
            phi = np.arctan2(v[:, 1], v[:, 0])
            psi_k[k] = np.mean(np.cos(6.0 * phi) + 1j * np.sin(6.0 * phi))
    return psi_k.mean(), psi_k, counts


def empty_circle_edges(x, y):
    """Delaunay edges of a small point set in the plane by definition: the
    sides of every triangle whose circumcircle holds no other point inside
    (points in general position; O(n^4), for a few dozen points)."""
    p = np.stack([np.asarray(x, float), np.asarray(y, float)], axis=1)
    n = len(p)
    edges = set()
    for i in range(n):
        for j in range(i + 1, n):
            for m in range(j + 1, n):
                a, b, c = p[i], p[j], p[m]
                d = 2.0 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
                if abs(d) < 1e-12:
                    continue  # collinear: no circumcircle
                ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
                uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
                r2 = (a[0] - ux) ** 2 + (a[1] - uy) ** 2
                others = np.ones(n, bool)
                others[[i, j, m]] = False
                dist2 = (p[others, 0] - ux) ** 2 + (p[others, 1] - uy) ** 2
                if np.all(dist2 > r2):
                    edges.update({(i, j), (i, m), (j, m)})
    return edges


def autocorrelation(psi, max_lag):
    """C(dt) of eq. (tau) for dt = 0..max_lag: the real part of the mean of
    Psi*(t) Psi(t + dt) over the available t, divided by the mean of |Psi|^2."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = len(psi)
    den = np.mean(np.abs(psi) ** 2)
    return np.array([np.mean(np.conj(psi[:n - d]) * psi[d:]).real / den
                     for d in range(max_lag + 1)])


def tau_fit(c):
    """Decay time of C(dt) ~ exp(-dt / tau): least squares of ln C(dt) = -dt / tau
    through the origin, over dt = 1, 2, ... while C(dt) > exp(-2)."""
    d, lc = [], []
    for lag in range(1, len(c)):
        if not c[lag] > np.exp(-2.0):
            break
        d.append(float(lag))
        lc.append(np.log(c[lag]))
    if not d:
        return None
    d = np.array(d)
    lc = np.array(lc)
    return -float(np.sum(d * d) / np.sum(d * lc))


def planar_neighbours(px, py, centre):
    """Delaunay neighbours of point `centre` of a planar patch (offsets from it),
    for sampling a large periodic system: the patch holds every disk within
    some radius R of the centre (unwrapped), and the result is that of the
    whole system when every triangle at the centre has its circumcircle
    inside the patch's disk of radius R, which is checked."""
    from scipy.spatial import Delaunay
    p = np.stack([np.asarray(px, float), np.asarray(py, float)], axis=1)
    R = np.sqrt(np.max(np.sum((p - p[centre]) ** 2, axis=1)))
    tri = Delaunay(p)
    s = tri.simplices[np.any(tri.simplices == centre, axis=1)]
    a, b, c = p[s[:, 0]], p[s[:, 1]], p[s[:, 2]]
    d = 2.0 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
    aa, bb, cc = (a * a).sum(1), (b * b).sum(1), (c * c).sum(1)
    ux = (aa * (b[:, 1] - c[:, 1]) + bb * (c[:, 1] - a[:, 1]) + cc * (a[:, 1] - b[:, 1])) / d
    uy = (aa * (c[:, 0] - b[:, 0]) + bb * (a[:, 0] - c[:, 0]) + cc * (b[:, 0] - a[:, 0])) / d
    r = np.sqrt((a[:, 0] - ux) ** 2 + (a[:, 1] - uy) ** 2)
    dc = np.sqrt((ux - p[centre, 0]) ** 2 + (uy - p[centre, 1]) ** 2)
    if np.any(dc + r > 0.999 * R):
        raise ValueError("patch too small for the Delaunay triangles at its centre")
    indptr, indices = tri.vertex_neighbor_vertices
    nb = indices[indptr[centre]:indptr[centre + 1]]
    return p[nb] - p[centre]
