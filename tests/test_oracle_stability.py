"""Von Neumann stability of the oracle's step, the basis of the library's Courant limits.

On a uniform periodic grid the step is a convolution: every cell applies the same stencil S
(a matrix over the field components per neighbour offset) to its neighbours.  A Fourier mode
v e^{i k.x} is then multiplied by the symbol G(k) = sum_offsets S(offset) e^{i k.offset}, and
the step is stable when no eigenvalue of G(k) exceeds 1 in modulus for any k.  The stencil is
read off the probed linear map (oracle/gks_linear.py) of one step on a 7-cell periodic grid:
the step reaches two cells in each direction, so a 7-cell period separates every offset.

What these runs fix (each is also a limit that gks_init_mesh enforces):
  * 2D, (Ez, Hx, Hy): stable up to c dt / h = 0.5 for every tau;
  * 2D with psi coupled (gamma = 1): stable at 0.42, a mode gains 11% per step at 0.5;
  * 3D, six fields: stable at 1/3 as tau -> 0; at tau = 0.01 dt a mode gains about 2e-5 per
    step there, and in the collisionless limit modes gain 6e-3 per step at 0.3;
  * 3D with phi and psi coupled (chi = gamma = 1): stable at 0.3, 2.6% per step at 1/3.
"""
import itertools

import numpy as np
import pytest

from oracle import gks_linear as GL
from oracle import gks_oracle as O

N = 7


def symbol_radius(dim, nu, tau_hat, phm, nk):
    """Largest |eigenvalue| of G(k) over an nk^dim grid of wavenumbers in [-pi, pi)^dim."""
    mesh = O.cart2d(N, N, bc=(0,) * 4) if dim == 2 else O.cart3d(N, N, N, bc=(0,) * 6)
    dt = nu / N
    L = GL.LinearStep(mesh, dt, tau_hat * dt, phm=phm)
    A = L.A.tocsr()
    nc, nk_f = mesh.ncells, len(L.comps)
    centre = (N // 2,) * dim

    def cell(p):
        return p[0] + N * p[1] if dim == 2 else p[0] + N * (p[1] + N * p[2])

    c0 = cell(centre)
    S = {}
    nnz = 0
    for off in itertools.product(range(-2, 3), repeat=dim):
        cc = cell(tuple(c + o for c, o in zip(centre, off)))
        M = np.array([[A[a * nc + c0, b * nc + cc] for b in range(nk_f)] for a in range(nk_f)])
        nnz += int(np.count_nonzero(M))
        S[off] = M
    # every entry of the centre cell's rows lies within two cells (no aliasing on 7 cells)
    assert nnz == sum(A[a * nc + c0].nnz for a in range(nk_f))
    ks = np.linspace(-np.pi, np.pi, nk, endpoint=False)
    K = np.stack(np.meshgrid(*([ks] * dim), indexing="ij"), -1).reshape(-1, dim)
    G = np.zeros((K.shape[0], nk_f, nk_f), complex)
    for off, M in S.items():
        G += np.exp(1j * (K @ np.array(off, dtype=float)))[:, None, None] * M
    return float(np.abs(np.linalg.eigvals(G)).max())


STABLE = 1.0 + 1e-12


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, 1.0, np.inf])
def test_2d_maxwell_stable_at_one_half(tau_hat):
    assert symbol_radius(2, 0.5, tau_hat, None, 64) <= STABLE


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, 1.0])
def test_2d_phm_stable_at_the_library_limit(tau_hat):
    assert symbol_radius(2, 0.42, tau_hat, (0.0, 1.0), 64) <= STABLE


def test_2d_phm_grows_at_one_half():
    """gamma = 1 at c dt / h = 0.5 and tau = 0.01 dt: a mode gains 11% per step."""
    r = symbol_radius(2, 0.5, 0.01, (0.0, 1.0), 64)
    assert 1.10 < r < 1.12


def test_3d_maxwell_at_one_third():
    """Stable at 1/3 as tau -> 0; weak growth at tau = 0.01 dt (about 2e-5 per step)."""
    assert symbol_radius(3, 1.0 / 3.0, 0.0, None, 24) <= STABLE
    r = symbol_radius(3, 1.0 / 3.0, 0.01, None, 24)
    assert 1e-6 < r - 1.0 < 1e-4


def test_3d_collisionless_grows_below_the_limit():
    """The free-transport part of the D3Q4 flux grows at any Courant number tried (6e-3 per step
    at 0.3 as tau -> infinity); the library guards it only through unstable_growth."""
    r = symbol_radius(3, 0.3, np.inf, None, 24)
    assert 3e-3 < r - 1.0 < 1e-2


@pytest.mark.parametrize("tau_hat", [0.0, 0.01])
def test_3d_phm_stable_at_the_library_limit(tau_hat):
    assert symbol_radius(3, 0.3, tau_hat, (1.0, 1.0), 24) <= STABLE


def test_3d_phm_grows_at_one_third():
    r = symbol_radius(3, 1.0 / 3.0, 0.01, (1.0, 1.0), 24)
    assert 1.02 < r < 1.03
