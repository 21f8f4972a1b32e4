"""Seeded synthetic inputs: gauge links, spinor sources, gauge transformations,
algebra directions.

This module holds no arithmetic of the Dirac operator, the representations or
the solver; it only draws inputs.  Both the HIP path and the CPU oracle
consume what it returns.

Recipes
-------
haar_links(dims, N, seed)
    Haar-random SU(N) per link: QR of a complex Gaussian matrix (Re, Im ~
    N(0, 1/2)), Q times the phases of diag(R) (Mezzadri's recipe), then the
    determinant is divided out with its principal N-th root, as in the
    Gram-Schmidt-then-det-fix SU(N) projection of Sec. 7.6.4.
expH_links(dims, N, eps, seed)
    U = exp(i eps H) per link with H Gaussian traceless Hermitian, distributed
    as sum_a h_a T^a with h_a ~ N(0,1) and tr T^a T^b = delta/2: off-diagonal
    entries with Re, Im ~ N(0, 1/4), diagonal ~ N(0, 1/2) projected to zero
    trace.  The exponential is taken through eigh.
gaussian_spinor(shape, seed)
    complex Gaussian, Re, Im ~ N(0, 1/2), so E|z|^2 = 1.
point_sources(dims, d, k)
    delta at the origin in spin k mod 4 and colour k // 4.

Shapes: links (T, X, Y, Z, 4, N, N) complex128; spinors (..., T, X, Y, Z, 4, d)
or half fields (..., V/2, 4, d).
"""
import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def _complex_gauss(rng, shape, var):
    s = np.sqrt(var)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


def haar_su_n(n_mat, N, rng):
    """n_mat Haar-random SU(N) matrices, array (n_mat, N, N)."""
    Z = _complex_gauss(rng, (n_mat, N, N), 0.5)
    Q, R = np.linalg.qr(Z)
    diag = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (diag / np.abs(diag))[:, None, :]
    det = np.linalg.det(Q)
    root = np.exp(1j * np.angle(det) / N)
    return Q / root[:, None, None]


def haar_links(dims, N, seed):
    rng = _rng(seed)
    V = int(np.prod(dims))
    return haar_su_n(V * 4, N, rng).reshape(tuple(dims) + (4, N, N))


def gaussian_traceless_hermitian(n_mat, N, rng):
    """Hermitian traceless H distributed as sum_a h_a T^a, h_a ~ N(0, 1)."""
    A = _complex_gauss(rng, (n_mat, N, N), 0.25)
    upper = np.triu(A, k=1)
    H = upper + np.conj(np.swapaxes(upper, -1, -2))
    g = rng.normal(0.0, np.sqrt(0.5), (n_mat, N))
    g = g - g.mean(axis=1, keepdims=True)
    idx = np.arange(N)
    H[:, idx, idx] = g
    return H


def expH_su_n(n_mat, N, eps, rng, chunk=1 << 20):
    out = np.empty((n_mat, N, N), dtype=np.complex128)
    for s in range(0, n_mat, chunk):
        e = min(n_mat, s + chunk)
        H = gaussian_traceless_hermitian(e - s, N, rng)
        w, V = np.linalg.eigh(H)
        out[s:e] = np.einsum('nij,nj,nkj->nik', V, np.exp(1j * eps * w), np.conj(V))
    return out


def expH_links(dims, N, eps, seed):
    rng = _rng(seed)
    V = int(np.prod(dims))
    return expH_su_n(V * 4, N, eps, rng).reshape(tuple(dims) + (4, N, N))


def expH_links_torch(dims, N, eps, seed, device='cuda'):
    """The exp(i eps H) recipe drawn with torch's seeded generator on `device`
    (for lattices whose links are too many for a host-side eigendecomposition):
    same distribution of H, exponential by torch.linalg.matrix_exp."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    shape = tuple(dims) + (4, N, N)
    re = torch.randn(shape, dtype=torch.float64, device=device, generator=g) * 0.5
    im = torch.randn(shape, dtype=torch.float64, device=device, generator=g) * 0.5
    A = torch.complex(re, im)
    upper = torch.triu(A, diagonal=1)
    H = upper + upper.conj().transpose(-1, -2)
    diag = torch.randn(tuple(dims) + (4, N), dtype=torch.float64, device=device, generator=g) * (0.5 ** 0.5)
    diag = diag - diag.mean(dim=-1, keepdim=True)
    H = H + torch.diag_embed(diag.to(torch.complex128))
    del A, upper, re, im
    return torch.linalg.matrix_exp(1j * eps * H)


def unit_links(dims, N):
    U = np.zeros(tuple(dims) + (4, N, N), dtype=np.complex128)
    idx = np.arange(N)
    U[..., idx, idx] = 1.0
    return U


def gaussian_spinor(shape, seed):
    return _complex_gauss(_rng(seed), tuple(shape), 0.5)


def point_sources(dims, d, nsrc):
    """nsrc point sources at the origin: source k sits in spin k % 4, colour k // 4."""
    psi = np.zeros((nsrc,) + tuple(dims) + (4, d), dtype=np.complex128)
    for k in range(nsrc):
        psi[(k, 0, 0, 0, 0, k % 4, k // 4)] = 1.0
    return psi


def gauge_transform(dims, N, seed):
    """Haar-random g(x) per site, array (T, X, Y, Z, N, N)."""
    rng = _rng(seed)
    V = int(np.prod(dims))
    return haar_su_n(V, N, rng).reshape(tuple(dims) + (N, N))


def algebra_directions(dims, N, seed):
    """Gaussian algebra components omega^a_mu(x), array (T, X, Y, Z, 4, N^2-1)."""
    rng = _rng(seed)
    return rng.normal(0.0, 1.0, tuple(dims) + (4, N * N - 1))


# Configurations of the benchmark and parity suite.  Each entry names the
# workload by what it is; the link recipe, seed and mass are fixed here.
CONFIGS = {
    'su2_fund_4x4x4x4': dict(N=2, rep='FUND', dims=(4, 4, 4, 4), m0=-0.2, links='haar',
                             seed=1000, bc=(-1, 1, 1, 1)),
    'su3_fund_32x32x32x32': dict(N=3, rep='FUND', dims=(32, 32, 32, 32), m0=-0.4, links='expH',
                                 eps=0.3, seed=1001, bc=(-1, 1, 1, 1)),
    'su4_2as_96x48x48x48': dict(N=4, rep='2AS', dims=(96, 48, 48, 48), m0=-0.3, links='expH',
                                eps=0.3, seed=1002, bc=(-1, 1, 1, 1)),
    'su3_sym_48x24x24x24': dict(N=3, rep='SYM', dims=(48, 24, 24, 24), m0=-0.4, links='expH',
                                eps=0.3, seed=1003, bc=(-1, 1, 1, 1), nrhs=12),
    'su2_adj_32x16x16x16': dict(N=2, rep='ADJ', dims=(32, 16, 16, 16), m0=-1.1, links='expH',
                                eps=0.3, seed=1004, bc=(-1, 1, 1, 1)),
}


def links_for(cfg):
    if cfg['links'] == 'haar':
        return haar_links(cfg['dims'], cfg['N'], cfg['seed'])
    return expH_links(cfg['dims'], cfg['N'], cfg['eps'], cfg['seed'])
