"""Exact solutions of the TM Maxwell system (c = eps = mu = 1) used to pin the oracle.

TEST INFRASTRUCTURE ONLY (imported by the tests alone).

  * plane wave (Sec. 5.1 generalised to any wave vector k = 2 pi (m, n)):
        Ez = cos(k.x - |k| t),  Hx = (k_y/|k|) cos(.),  Hy = -(k_x/|k|) cos(.)
    The paper's case Ez = cos 2 pi (x - t), B_y = -Ez is m = 1, n = 0.
  * cavity eigenmode (Sec. 5.2), omega0 = sqrt(2) a:
        Ez = sin(ax) sin(ay) cos(w t), Hx = -(a/w) sin(ax) cos(ay) sin(w t),
        Hy = (a/w) cos(ax) sin(ay) sin(w t)
  * periodic Gaussian on the unit square, H = 0 at t = 0, from its Fourier series
        Ez = sum_k E_k cos(|k| t) e^{ik.x},  E_k = 2 pi w^2 exp(-w^2 |k|^2 / 2) e^{-ik.x_c}
        Hx = -sum_k E_k (i k_y/|k|) sin(|k| t) e^{ik.x},  Hy = +sum_k E_k (i k_x/|k|) sin(|k| t) e^{ik.x}
Each satisfies dEz/dt = dHy/dx - dHx/dy, dHx/dt = -dEz/dy, dHy/dt = dEz/dx.
"""
from __future__ import annotations

import numpy as np


def plane_wave_tm(x, y, t, m=1, n=0):
    kx, ky = 2 * np.pi * m, 2 * np.pi * n
    k = np.hypot(kx, ky)
    ph = np.cos(kx * x + ky * y - k * t)
    return ph, (ky / k) * ph, -(kx / k) * ph


def cavity_tm(x, y, t, a=8 * np.pi):
    w = np.sqrt(2.0) * a
    ez = np.sin(a * x) * np.sin(a * y) * np.cos(w * t)
    hx = -(a / w) * np.sin(a * x) * np.cos(a * y) * np.sin(w * t)
    hy = (a / w) * np.cos(a * x) * np.sin(a * y) * np.sin(w * t)
    return ez, hx, hy


def gaussian_tm(x, y, t, xc, yc, w=0.05, kmax=40):
    """Periodic Gaussian exp(-|x - x_c|^2/(2 w^2)) summed over its periodic images, evolved
    exactly; truncation at |m|, |n| <= kmax (the dropped terms are below 1e-30 for w = 0.05)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ms = np.arange(-kmax, kmax + 1)
    kx = 2 * np.pi * ms
    # separable sums: e^{ik.x} = e^{i kx x} e^{i ky y}
    ex = np.exp(1j * np.multiply.outer(x.ravel(), kx))     # (P, K)
    ey = np.exp(1j * np.multiply.outer(y.ravel(), kx))
    KX, KY = np.meshgrid(kx, kx, indexing="ij")            # (K, K): [m, n]
    kk = np.hypot(KX, KY)
    E = 2 * np.pi * w * w * np.exp(-0.5 * w * w * kk ** 2) * np.exp(-1j * (KX * xc + KY * yc))
    c = np.cos(kk * t)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(kk > 0, np.sin(kk * t) / kk, 0.0)
    A_ez = E * c
    A_hx = -E * (1j * KY) * s
    A_hy = E * (1j * KX) * s
    out = []
    for A in (A_ez, A_hx, A_hy):
        v = np.einsum("pm,mn,pn->p", ex, A, ey)
        out.append(v.real.reshape(x.shape))
    return tuple(out)


def error_norms(num, ref):
    """L1 = mean |e|, L2 = sqrt(mean e^2), Linf = max |e|."""
    e = np.asarray(num) - np.asarray(ref)
    return float(np.mean(np.abs(e))), float(np.sqrt(np.mean(e * e))), float(np.max(np.abs(e)))
