"""FP64 reference of the surrogate network's layers (oracle; tests only).

The surrogate is not in the paper: it is a learned approximation of the map
I -> S_ph of eq. (integral) on a coarse grid, trained on pairs produced by the
FMM.  This module is the plain definition of every layer it uses, on arrays in
grid order [C, n, n, n] (batch as a leading list), written from the definitions
of cross-correlation, strided convolution, and their adjoints:

  conv3   y[o, z, y, x] = sum_{i, dz, dy, dx} w[o, i, dz+1, dy+1, dx+1] x[i, z+dz, y+dy, x+dx]
          (3x3x3, zero padding, stride 1)
  down2   y[o, Z] = sum_{i, p} w[o, i, p] x[i, 2Z + p]        (2x2x2, stride 2)
  up2     y[o, 2Z + p] = sum_i w[o, i, p] x[i, Z]            (transposed 2x2x2, stride 2)
  point   y[o] = sum_i w[o, i] x[i]                          (1x1x1)
  leaky   y = x for x > 0, alpha x otherwise
  loss    L = ||y - t||^2 / ||t||^2  (squared relative L2 per sample, mean over samples)
  adam    m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
          w -= lr * (m / (1-b1^k)) / (sqrt(v / (1-b2^k)) + eps)
"""
import numpy as np


def _shifted(x, dz, dy, dx):
    """x[..., z+dz, y+dy, x+dx] with zeros outside (last three axes)."""
    out = np.zeros_like(x)
    n = x.shape[-3:]
    src = tuple(slice(max(0, d), m + min(0, d)) for d, m in zip((dz, dy, dx), n))
    dst = tuple(slice(max(0, -d), m + min(0, -d)) for d, m in zip((dz, dy, dx), n))
    out[(Ellipsis,) + dst] = x[(Ellipsis,) + src]
    return out


def conv3(x, w):
    """x [ci, n, n, n], w [co, ci, 3, 3, 3] -> [co, n, n, n]."""
    y = np.zeros((w.shape[0],) + x.shape[1:])
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = _shifted(x, dz, dy, dx)
                y += np.einsum("oi,izyx->ozyx", w[:, :, dz + 1, dy + 1, dx + 1], xs)
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 with respect to x and w given dL/dy."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                wt = w[:, :, dz + 1, dy + 1, dx + 1]
                # y(z) uses x(z + d): x(z') receives from y(z' - d)
                gx += np.einsum("oi,ozyx->izyx", wt, _shifted(gy, -dz, -dy, -dx))
                gw[:, :, dz + 1, dy + 1, dx + 1] = np.einsum("ozyx,izyx->oi", gy, _shifted(x, dz, dy, dx))
    return gx, gw


def _blocks(x):
    """[c, 2m, 2m, 2m] -> [c, m, m, m, 2, 2, 2] with the last axes the parity p."""
    c, n = x.shape[0], x.shape[1]
    m = n // 2
    return x.reshape(c, m, 2, m, 2, m, 2).transpose(0, 1, 3, 5, 2, 4, 6)


def _unblocks(b):
    c, m = b.shape[0], b.shape[1]
    return b.transpose(0, 1, 4, 2, 5, 3, 6).reshape(c, 2 * m, 2 * m, 2 * m)


def down2(x, w):
    """x [ci, 2m, ..], w [co, ci, 2, 2, 2] -> [co, m, m, m]."""
    return np.einsum("oipqr,iZYXpqr->oZYX", w, _blocks(x))


def down2_backward(x, w, gy):
    gx = _unblocks(np.einsum("oipqr,oZYX->iZYXpqr", w, gy))
    gw = np.einsum("oZYX,iZYXpqr->oipqr", gy, _blocks(x))
    return gx, gw


def up2(x, w):
    """x [ci, m, m, m], w [co, ci, 2, 2, 2] -> [co, 2m, 2m, 2m]."""
    return _unblocks(np.einsum("oipqr,iZYX->oZYXpqr", w, x))


def up2_backward(x, w, gy):
    gb = _blocks(gy)
    gx = np.einsum("oipqr,oZYXpqr->iZYX", w, gb)
    gw = np.einsum("oZYXpqr,iZYX->oipqr", gb, x)
    return gx, gw


def point(x, w):
    return np.einsum("oi,izyx->ozyx", w, x)


def point_backward(x, w, gy):
    return np.einsum("oi,ozyx->izyx", w, gy), np.einsum("ozyx,izyx->oi", gy, x)


def leaky(x, alpha):
    return np.where(x > 0, x, alpha * x)


def leaky_backward(x, alpha, gy):
    return np.where(x > 0, gy, alpha * gy)


def rel_l2_loss(y, t):
    """Mean over samples of ||y - t||^2 / ||t||^2 and its gradient (lists of arrays)."""
    n = len(y)
    L = 0.0
    g = []
    for yi, ti in zip(y, t):
        d2 = float(np.sum(ti * ti))
        L += float(np.sum((yi - ti) ** 2)) / d2 / n
        g.append(2.0 * (yi - ti) / d2 / n)
    return L, g


def adam(w, g, m, v, k, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step number k >= 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def coarsen2(f):
    """2x2x2 block means of an [n, n, n] field (n even)."""
    n = f.shape[0] // 2
    return f.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))


def upsample2(c):
    """Trilinear interpolation of an m^3 field of cell-centre values to the cell
    centres of the (2m)^3 refinement; fine centre i sits at coarse coordinate
    (i + 1/2)/2 - 1/2, clamped to [0, m-1] (constant extension at the faces)."""
    m = c.shape[0]
    x = np.clip((np.arange(2 * m) + 0.5) / 2 - 0.5, 0, m - 1)
    i0 = np.floor(x).astype(int)
    i1 = np.minimum(i0 + 1, m - 1)
    w = x - i0
    out = c
    for ax in range(3):
        a = np.take(out, i0, axis=ax)
        b = np.take(out, i1, axis=ax)
        shape = [1, 1, 1]
        shape[ax] = -1
        out = a * (1 - w.reshape(shape)) + b * w.reshape(shape)
    return out


def neighbourhood27(f):
    """[n, n, n] -> [32, n, n, n]: channel (dz+1)*9 + (dy+1)*3 + (dx+1) holds f at
    offset (dz, dy, dx) (zero outside the grid), channels 27..31 zero."""
    out = np.zeros((32,) + f.shape)
    c = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out[c] = _shifted(f[None], dz, dy, dx)[0]
                c += 1
    return out
