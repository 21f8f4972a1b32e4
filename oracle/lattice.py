"""Lattice geometry for the oracle.

Conventions (paper Sec. 2.1 and Sec. 5.3.3):
  * a site is (t, x, y, z); direction mu = 0 is time; fields are NumPy arrays
    whose first four axes are (T, X, Y, Z);
  * the lexicographic index is ((t*X + x)*Y + y)*Z + z (C order of the array);
  * a site is even when (t + x + y + z) mod 2 == 0, odd otherwise;
  * a half field of parity p lists the sites of parity p in increasing
    lexicographic order;
  * boundary conditions (Sec. 6.3.1): bc[mu] = +1 (periodic) or -1
    (antiperiodic) for the fermion field, psi(x + L_mu e_mu) = bc[mu] psi(x).
    Gauge links are always periodic.
"""
import numpy as np


def volume(dims):
    return int(np.prod(dims))


def coordinates(dims):
    """(V, 4) integer array: row i holds the (t, x, y, z) of lexicographic site i."""
    V = volume(dims)
    return np.stack(np.unravel_index(np.arange(V), tuple(dims)), axis=1)


def parity_field(dims):
    """Array of shape dims holding (t+x+y+z) mod 2 (Sec. 5.3.3)."""
    c = coordinates(dims)
    return (c.sum(axis=1) % 2).reshape(tuple(dims))


def parity_sites(dims, p):
    """Lexicographic indices of the sites of parity p, in increasing order."""
    return np.flatnonzero(parity_field(dims).ravel() == p)


def to_half(full, dims, p):
    """Restrict a full field (leading axes T,X,Y,Z) to the sites of parity p."""
    V = volume(dims)
    flat = full.reshape((V,) + full.shape[4:])
    return flat[parity_sites(dims, p)].copy()


def from_half(half, dims, p):
    """Embed a half field of parity p into a full field that is zero elsewhere."""
    V = volume(dims)
    flat = np.zeros((V,) + half.shape[1:], dtype=half.dtype)
    flat[parity_sites(dims, p)] = half
    return flat.reshape(tuple(dims) + half.shape[1:])


def shift_fwd(f, mu, bc):
    """g(x) = f(x + mu), with the fermion boundary phase bc[mu] on the wrap."""
    g = np.roll(f, -1, axis=mu)
    if bc[mu] != 1:
        idx = [slice(None)] * g.ndim
        idx[mu] = -1                       # sites with x_mu = L_mu - 1 read f(0)
        g[tuple(idx)] *= bc[mu]
    return g


def shift_bwd(f, mu, bc):
    """g(x) = f(x - mu), with the fermion boundary phase bc[mu] on the wrap."""
    g = np.roll(f, 1, axis=mu)
    if bc[mu] != 1:
        idx = [slice(None)] * g.ndim
        idx[mu] = 0                        # sites with x_mu = 0 read f(L_mu - 1)
        g[tuple(idx)] *= bc[mu]
    return g


def link_bwd(U, mu):
    """U(x - mu, mu) for every x (links are periodic)."""
    return np.roll(U[..., mu, :, :], 1, axis=mu)


def neighbour(coord, mu, step, dims):
    """Coordinates of coord + step*mu (step = +1 or -1) and whether the hop wraps.

    coord is an (n, 4) integer array.  Returns (coords, wrapped)."""
    c = np.array(coord, copy=True)
    c[:, mu] += step
    wrapped = (c[:, mu] < 0) | (c[:, mu] >= dims[mu])
    c[:, mu] %= dims[mu]
    return c, wrapped
