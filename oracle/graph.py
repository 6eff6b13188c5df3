"""Atomic graphs: periodic radius graph, ghost shells and subdomains.

TEST INFRASTRUCTURE (see oracle/__init__.py).

Section 2: atoms closer than r_c are joined by an edge.  The edge v<-w
carries the displacement r_vw = r_w - r_v (section 3.1, before eq 5); the
receiver is v and the sender is w.  Under periodic boundary conditions the
sender may be any periodic image r_w + n H (n integer, H the cell with
lattice vectors as rows), including images of the receiver itself.

Section 3.1: a subdomain evaluates its own atoms; neighbours owned by other
subdomains (or periodic images) are "ghost" atoms that receive positions,
species and node features from their owners.  Here a ghost is a pair
(owner atom, integer image shift).

Everything here is brute force over all pairs and image shifts, in float64.
"""
from __future__ import annotations

import math

import numpy as np


def perp_widths(cell: np.ndarray) -> np.ndarray:
    vol = abs(np.linalg.det(cell))
    a, b, c = cell
    return np.array([vol / np.linalg.norm(np.cross(b, c)),
                     vol / np.linalg.norm(np.cross(c, a)),
                     vol / np.linalg.norm(np.cross(a, b))])


def wrap(pos: np.ndarray, cell: np.ndarray, pbc=(True, True, True)) -> np.ndarray:
    """f = R H^-1, f <- f - floor(f) on periodic axes, R = f H."""
    f = pos @ np.linalg.inv(cell)
    for a in range(3):
        if pbc[a]:
            f[:, a] -= np.floor(f[:, a])
            f[:, a] = np.where(f[:, a] >= 1.0, 0.0, f[:, a])
    return f @ cell


def _image_range(cell, pbc, reach):
    w = perp_widths(cell)
    return [int(math.ceil(reach / w[a])) if pbc[a] else 0 for a in range(3)]


def _kdtree_edges(pos, cell, r_cut):
    """Orthorhombic cell wider than 2 r_c on every axis: each pair has at most one image
    within r_c, found by a periodic kd-tree (scipy); shifts from the minimum image."""
    from scipy.spatial import cKDTree
    L = np.diag(cell).copy()
    f = pos / L
    f -= np.floor(f)
    p = np.minimum(f * L, np.nextafter(L, 0))
    pairs = cKDTree(p, boxsize=L).query_pairs(r_cut, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    d = pos[j] - pos[i]
    n = -np.round(d / L).astype(np.int64)
    dd = d + n * L
    r2 = np.einsum("ij,ij->i", dd, dd)
    keep = (r2 < r_cut * r_cut) & (r2 > 0)
    i, j, n = i[keep], j[keep], n[keep]
    recv = np.concatenate([i, j])
    send = np.concatenate([j, i])
    shift = np.concatenate([n, -n])
    order = np.lexsort((shift[:, 2], shift[:, 1], shift[:, 0], send, recv))
    return recv[order], send[order], shift[order]


def periodic_edges(pos: np.ndarray, cell: np.ndarray, r_cut: float, pbc=(True, True, True),
                   chunk: int = 256):
    """All (i, j, n) with 0 < |R_j + n H - R_i| < r_cut.

    Returns recv [E], send [E], shift [E, 3] (int), sorted by receiver, then
    sender, then shift.  Brute force over all pairs and image shifts, except for
    large orthorhombic cells (every side > 2 r_c, > 2000 atoms), where a periodic
    kd-tree gives the same set (pinned against brute force in the tests).
    """
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    if (all(pbc) and np.allclose(cell, np.diag(np.diag(cell)), atol=0) and pos.shape[0] > 2000
            and np.all(np.diag(cell) > 2 * r_cut)):
        return _kdtree_edges(pos, cell, r_cut)
    nr = _image_range(cell, pbc, r_cut)
    shifts = np.array([(a, b, c) for a in range(-nr[0], nr[0] + 1)
                       for b in range(-nr[1], nr[1] + 1)
                       for c in range(-nr[2], nr[2] + 1)], dtype=np.int64)
    svec = shifts @ cell
    rc2 = r_cut * r_cut
    N = pos.shape[0]
    out_r, out_s, out_n = [], [], []
    for i0 in range(0, N, chunk):
        pi = pos[i0:i0 + chunk]
        for k, sv in enumerate(svec):
            d = pos[None, :, :] + sv[None, None, :] - pi[:, None, :]
            r2 = np.einsum("ijk,ijk->ij", d, d)
            ii, jj = np.nonzero((r2 < rc2) & (r2 > 0.0))
            out_r.append(ii + i0)
            out_s.append(jj)
            out_n.append(np.repeat(shifts[k][None], len(ii), axis=0))
    recv = np.concatenate(out_r)
    send = np.concatenate(out_s)
    shift = np.concatenate(out_n).reshape(-1, 3)
    order = np.lexsort((shift[:, 2], shift[:, 1], shift[:, 0], send, recv))
    return recv[order], send[order], shift[order]


def domain_points(frac: np.ndarray, lo, hi, delta, pbc=(True, True, True)):
    """Points of the extended subdomain [lo - delta, hi + delta) in fractional space.

    Returns (local_ids, ghost_owner, ghost_shift): local atoms are those with
    fractional coordinates in [lo, hi) (shift 0); ghosts are every other image
    (atom j, shift n) inside the extended box, ordered by owner then shift.
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    delta = np.asarray(delta, float)
    rng = [range(-int(math.ceil(delta[a])) - 1, int(math.ceil(delta[a])) + 2) if pbc[a] else range(0, 1)
           for a in range(3)]
    local = np.nonzero(np.all((frac >= lo) & (frac < hi), axis=1))[0]
    is_local = np.zeros(frac.shape[0], bool)
    is_local[local] = True
    lo_e = np.where(np.asarray(pbc), lo - delta, -np.inf)
    hi_e = np.where(np.asarray(pbc), hi + delta, np.inf)
    owners, shifts = [], []
    for a in rng[0]:
        for b in rng[1]:
            for c in rng[2]:
                n = np.array([a, b, c])
                f = frac + n
                ok = np.all((f >= lo_e) & (f < hi_e), axis=1)
                if a == 0 and b == 0 and c == 0:
                    ok &= ~is_local
                idx = np.nonzero(ok)[0]
                owners.append(idx)
                shifts.append(np.repeat(n[None], len(idx), axis=0))
    owners = np.concatenate(owners)
    shifts = np.concatenate(shifts).reshape(-1, 3)
    order = np.lexsort((shifts[:, 2], shifts[:, 1], shifts[:, 0], owners))
    owners, shifts = owners[order], shifts[order]
    return local, owners.astype(np.int64), shifts.astype(np.int64)


def domain_edges(pos_ext: np.ndarray, n_local: int, r_cut: float, chunk: int = 256):
    """Edges with a local receiver (rows < n_local) and any extended sender."""
    rc2 = r_cut * r_cut
    out_r, out_s = [], []
    for i0 in range(0, n_local, chunk):
        pi = pos_ext[i0:min(i0 + chunk, n_local)]
        d = pos_ext[None, :, :] - pi[:, None, :]
        r2 = np.einsum("ijk,ijk->ij", d, d)
        ii, jj = np.nonzero((r2 < rc2) & (r2 > 0.0))
        out_r.append(ii + i0)
        out_s.append(jj)
    recv = np.concatenate(out_r)
    send = np.concatenate(out_s)
    order = np.lexsort((send, recv))
    return recv[order], send[order]


def ghost_shell(pos_wrapped: np.ndarray, cell: np.ndarray, r_cut: float, skin: float = 0.0,
                pbc=(True, True, True)):
    """One subdomain (the whole cell) plus a ghost shell of width r_c + skin.

    Returns dict(local, ghost_owner, ghost_shift, recv, send) with senders
    indexing [locals..., ghosts...].
    """
    frac = pos_wrapped @ np.linalg.inv(cell)
    delta = (r_cut + skin) / perp_widths(cell)
    local, owner, shift = domain_points(frac, [0, 0, 0], [1, 1, 1], delta, pbc)
    assert len(local) == pos_wrapped.shape[0]
    pos_ext = np.concatenate([pos_wrapped[local], pos_wrapped[owner] + shift @ cell])
    recv, send = domain_edges(pos_ext, len(local), r_cut)
    return dict(local=local, ghost_owner=owner, ghost_shift=shift, recv=recv, send=send)


def subdomains(pos_wrapped: np.ndarray, cell: np.ndarray, r_cut: float, splits=(2, 1, 1),
               skin: float = 0.0):
    """Regular grid of subdomains in fractional space, each with its own shell.

    Returns a list of dicts like ghost_shell(); `local` and `ghost_owner` are
    global atom indices.
    """
    frac = pos_wrapped @ np.linalg.inv(cell)
    delta = (r_cut + skin) / perp_widths(cell)
    out = []
    for a in range(splits[0]):
        for b in range(splits[1]):
            for c in range(splits[2]):
                lo = np.array([a / splits[0], b / splits[1], c / splits[2]])
                hi = np.array([(a + 1) / splits[0], (b + 1) / splits[1], (c + 1) / splits[2]])
                local, owner, shift = domain_points(frac, lo, hi, delta)
                pos_ext = np.concatenate([pos_wrapped[local], pos_wrapped[owner] + shift @ cell])
                recv, send = domain_edges(pos_ext, len(local), r_cut)
                out.append(dict(local=local, ghost_owner=owner, ghost_shift=shift,
                                recv=recv, send=send))
    return out
