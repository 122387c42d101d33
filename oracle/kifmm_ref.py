"""Plain FP64 kernel-independent FMM on a uniform grid (oracle; tests only).

Follows Section 3 step by step, in the paper's density form, with no fusion of
operators: every translation first evaluates a check potential and then solves
for an equivalent density with the truncated-SVD pseudo-inverse.

  tree      complete octree over an n^3 grid, leaves of ell^3 cells
            (tree construction step of the algorithm outline)
  upward    leaves: check potential q^{B,u} from the sources, eq. (s2m);
            parents: q^{P,u} from the children's densities, eq. (m2m);
            then phi^{B,u} = pinv(G(x^{B,u}, y^{B,u})) q^{B,u}
  downward  levels 2..D: q^{B,d} gets the densities of the boxes A in the
            interaction list of B (children of the neighbours of P(B) that are
            not adjacent to B), eq. (m2l), and the parent's downward density,
            eq. (l2l); then phi^{B,d} = pinv(G(x^{B,d}, y^{B,d})) q^{B,d}
  targets   leaf B: the downward density evaluated at the cell centres plus the
            direct sum over the 27 leaves of the near range N(B), eq. (nearfar)

The pseudo-inverse is numpy.linalg.pinv with a relative cutoff: singular values
at or below rcond * s_max are dropped (the "original pseudo-inverse").

The matrices G(x^{B,d}, y^{A,u}) depend only on the level and the offset A - B,
so each one is formed once per level and offset and applied to all box pairs with
that offset; this reuses a matrix, it does not change the arithmetic.

Point sets.  The text fixes m0 points per cube edge (m0 = 6) but not the radii;
three layouts are provided, all in units of the box half-width r:
  'paper'   one surface each: y^u at 1.05 r, x^u at 2.95 r, y^d at 2.95 r,
            x^d at 1.05 r (m0 points per edge on every surface)
  'single'  y^u: m0 surface at 1.05 r; x^u: surfaces at 2.95 r, 4 r and 6 r with
            `check_edge` points per edge; y^d: m0 surface at 2.95 r; x^d: a
            check_edge^3 lattice filling [-1.05 r, 1.05 r]^3
  'nested'  as 'single' but y^u adds an m0 surface at 0.55 r and y^d adds an
            m0 surface at 4 r
  'lattice' y^u and x^d: the full m0^3 lattice filling [-R r, R r]^3 (R =
            lattice_radius, 1.2 by default); x^u as in 'single'; y^d as in 'nested'.  Equivalent points and M2L check points
            then lie on lattices of one spacing, so each M2L matrix G(x^d, y^u + 2 r o)
            is a block of a 3-D convolution (the FFT form of M2L, Section 3 remark);
            here it is still applied as the plain matrix
"""
import itertools

import numpy as np

from . import kernel as _k

LAYOUTS = ("paper", "single", "nested", "lattice")


def cube_surface(m, rad):
    """Points of an m x m x m lattice on [-rad, rad]^3 that lie on its boundary."""
    t = np.linspace(-rad, rad, m)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    idx = np.stack(np.meshgrid(*(np.arange(m),) * 3, indexing="ij"), -1).reshape(-1, 3)
    on = ((idx == 0) | (idx == m - 1)).any(axis=1)
    return g[on]


def cube_lattice(m, rad):
    t = np.linspace(-rad, rad, m)
    return np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)


def point_sets(layout, m0, check_edge, r, lattice_radius=1.2):
    """(y_u, x_u, y_d, x_d) relative to the box centre for half-width r."""
    if layout == "paper":
        return (cube_surface(m0, 1.05 * r), cube_surface(m0, 2.95 * r),
                cube_surface(m0, 2.95 * r), cube_surface(m0, 1.05 * r))
    xu = np.vstack([cube_surface(check_edge, f * r) for f in (2.95, 4.0, 6.0)])
    xd = cube_lattice(check_edge, 1.05 * r)
    if layout == "single":
        return cube_surface(m0, 1.05 * r), xu, cube_surface(m0, 2.95 * r), xd
    if layout == "nested":
        yu = np.vstack([cube_surface(m0, 1.05 * r), cube_surface(m0, 0.55 * r)])
        yd = np.vstack([cube_surface(m0, 2.95 * r), cube_surface(m0, 4.0 * r)])
        return yu, xu, yd, xd
    if layout == "lattice":
        yd = np.vstack([cube_surface(m0, 2.95 * r), cube_surface(m0, 4.0 * r)])
        R = lattice_radius * r
        return cube_lattice(m0, R), xu, yd, cube_lattice(m0, R)
    raise ValueError(layout)


def gmat(X, Y, p_o2):
    """G(x_j, y_k) = K(|x_j - y_k|) for point sets that never coincide."""
    d = X[:, None, :] - Y[None, :, :]
    return _k.K(np.sqrt((d * d).sum(-1)), p_o2)


def _blocks(a, nb, ell):
    """(n,n,n) grid array -> (nb,nb,nb, ell^3), cells of each leaf in C order."""
    return a.reshape(nb, ell, nb, ell, nb, ell).transpose(0, 2, 4, 1, 3, 5).reshape(nb, nb, nb, -1)


def _unblocks(b, nb, ell):
    n = nb * ell
    return b.reshape(nb, nb, nb, ell, ell, ell).transpose(0, 3, 1, 4, 2, 5).reshape(n, n, n)


def _shift(arr, o):
    """out[B] = arr[B + o] where B + o is inside the box grid, else 0 (first 3 axes)."""
    n = arr.shape[0]
    out = np.zeros_like(arr)
    src, dst = [], []
    for d in o:
        src.append(slice(max(0, d), n + min(0, d)))
        dst.append(slice(max(0, -d), n + min(0, -d)))
    out[tuple(dst)] = arr[tuple(src)]
    return out


def evaluate(I, L, p_o2, ell, layout="nested", m0=6, check_edge=10, rcond=1e-10,
             prefactor=1.0, lattice_radius=1.2):
    """KIFMM approximation of S on an n^3 grid of cubic cells spanning [0, L]^3.

    I: (n,n,n) source values; returns S of the same shape (FP64).
    """
    I = np.asarray(I, dtype=np.float64)
    n = I.shape[0]
    assert I.shape == (n, n, n)
    h = L / n
    nb = n // ell
    assert nb * ell == n and nb & (nb - 1) == 0
    D = int(round(np.log2(nb)))
    q = I * (prefactor * h ** 3)
    qb = _blocks(q, nb, ell)

    # cell centres of a leaf relative to its centre
    t = (np.arange(ell) + 0.5) * h - 0.5 * ell * h
    P = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)

    # near field: the 27 leaves of N(B), eq. (nearfar); self value on the diagonal
    near = np.zeros_like(qb)
    for o in itertools.product((-1, 0, 1), repeat=3):
        M = gmat(P, P + np.array(o) * ell * h, p_o2) if any(o) else None
        if M is None:
            d = P[:, None, :] - P[None, :, :]
            R = np.sqrt((d * d).sum(-1))
            np.fill_diagonal(R, 1.0)
            M = _k.K(R, p_o2)
            np.fill_diagonal(M, _k.self_value(h, h, h, p_o2))
        near += _shift(qb, o) @ M.T
    if D < 2:
        return _unblocks(near, nb, ell)

    sets, pinv_u, pinv_d = {}, {}, {}
    for l in range(2, D + 1):
        r = L / 2 ** (l + 1)
        yu, xu, yd, xd = point_sets(layout, m0, check_edge, r, lattice_radius)
        sets[l] = (r, yu, xu, yd, xd)
        pinv_u[l] = np.linalg.pinv(gmat(xu, yu, p_o2), rcond=rcond)
        pinv_d[l] = np.linalg.pinv(gmat(xd, yd, p_o2), rcond=rcond)

    children = list(itertools.product((0, 1), repeat=3))

    # upward pass (post-order): eq. (s2m) at the leaves, eq. (m2m) above
    phi_u = {}
    r, yu, xu, _, _ = sets[D]
    q_check = qb @ gmat(xu, P, p_o2).T
    phi_u[D] = q_check @ pinv_u[D].T
    for l in range(D - 1, 1, -1):
        r, yu, xu, _, _ = sets[l]
        rc, yuc = sets[l + 1][0], sets[l + 1][1]
        nl = 2 ** l
        q_check = np.zeros((nl, nl, nl, xu.shape[0]))
        for c in children:
            centre = (np.array(c) - 0.5) * 2 * rc      # child centre minus parent centre
            q_check += phi_u[l + 1][c[0]::2, c[1]::2, c[2]::2] @ gmat(xu, yuc + centre, p_o2).T
        phi_u[l] = q_check @ pinv_u[l].T

    # downward pass (pre-order): eq. (m2l) from the interaction list, eq. (l2l)
    phi_d = {}
    for l in range(2, D + 1):
        r, yu, xu, yd, xd = sets[l]
        nl = 2 ** l
        q_check = np.zeros((nl, nl, nl, xd.shape[0]))
        if l > 2:
            yd_p = sets[l - 1][3]
            for c in children:
                centre = (np.array(c) - 0.5) * 2 * r   # parent centre is at -centre
                q_check[c[0]::2, c[1]::2, c[2]::2] += phi_d[l - 1] @ gmat(xd, yd_p - centre, p_o2).T
        idx = np.arange(nl)
        for o in itertools.product(range(-3, 4), repeat=3):
            if max(abs(v) for v in o) <= 1:
                continue
            # A = B + o is in the list of B when the parents of A and B are adjacent
            ok = [np.abs((idx + v) // 2 - idx // 2) <= 1 for v in o]
            ok = [m & (idx + v >= 0) & (idx + v < nl) for m, v in zip(ok, o)]
            mask = ok[0][:, None, None] & ok[1][None, :, None] & ok[2][None, None, :]
            if not mask.any():
                continue
            G = gmat(xd, yu + 2 * r * np.array(o), p_o2)
            src = _shift(phi_u[l], o)
            q_check[mask] += src[mask] @ G.T
        phi_d[l] = q_check @ pinv_d[l].T

    yd = sets[D][3]
    far = phi_d[D] @ gmat(P, yd, p_o2).T
    return _unblocks(near + far, nb, ell)
