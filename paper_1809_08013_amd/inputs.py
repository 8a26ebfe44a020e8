"""Seeded synthetic initial conditions for the two test problems of the paper.

This module is the single source of inputs for both the FP64 CPU oracle and the
HIP path. It holds none of the SPH step's arithmetic (no kernel, no density,
no forces, no neighbour search): only lattice placement, seeded random
sampling and the closed-form initial fields the paper prints.

* Rotating square patch (Sec. 5.1, "Rotating square patch"): a 2D square of
  side L rotating rigidly with v = (omega*y, -omega*x) (the rigid-rotation
  velocity equation of that subsection), extruded along z into a cube that is
  periodic in z, with the initial pressure given by the double sine series of
  that subsection.
* Evrard sphere (Sec. 5.1, "Evrard collapse"): density rho(r) = M/(2 pi R^2 r)
  inside R (the radial profile equation of that subsection) with R = M = 1,
  u0 = 0.05 and an ideal gas with gamma = 5/3.

All arrays are float64 (int32 for ids) in original-id order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SphParams",
    "SphIC",
    "square_patch",
    "square_patch_pressure",
    "evrard",
    "lattice_periodic",
    "random_cloud",
]


@dataclass
class SphParams:
    """Scalar physics constants shared by both paths.

    eos: 0 = weakly compressible Tait, 1 = ideal gas.
    kernel: 0 = M4 spline, 1 = Wendland C2, 2 = sinc of exponent sinc_n.
    gradient: 0 = kernel derivatives, 1 = integral approach (IAD).
    volume: 0 = standard volume elements m/rho, 1 = generalised volume
    elements with weights X = (m / rho_previous)^volume_p.
    The Tait exponent, eta^2, the Courant and force factors are the usual
    Monaghan (1992, 1994) choices; the paper leaves them open.
    """

    eos: int = 0
    rho0: float = 1.0
    c0: float = 50.0
    gamma_tait: float = 7.0
    gamma_gas: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    eta2: float = 0.01
    c_cfl: float = 0.3
    c_force: float = 0.25
    kernel: int = 0
    sinc_n: int = 5
    gradient: int = 0
    volume: int = 0
    volume_p: float = 0.7


@dataclass
class SphIC:
    """Particle state in original-id order plus the box it lives in."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    u: np.ndarray
    h: np.ndarray
    m: np.ndarray
    p_bg: np.ndarray
    id: np.ndarray
    lo: tuple
    hi: tuple
    periodic: tuple
    params: SphParams = field(default_factory=SphParams)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in
                ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "p_bg", "id")}

    def take(self, sel: np.ndarray) -> "SphIC":
        """Subset of particles (ids are kept)."""
        a = {k: np.ascontiguousarray(v[sel]) for k, v in self.arrays().items()}
        return SphIC(**a, lo=self.lo, hi=self.hi, periodic=self.periodic,
                     params=self.params, meta=dict(self.meta))


def square_patch_pressure(x: np.ndarray, y: np.ndarray, L: float = 1.0,
                          omega: float = 5.0, rho: float = 1.0,
                          kmax: int = 99) -> np.ndarray:
    """Initial pressure of the rotating square patch (Sec. 5.1 pressure series).

    The printed series is garbled; the reading used here is the double sine
    expansion that solves lap(P) = 2 rho omega^2 with P = 0 on the edges:
    only odd m, n >= 1 contribute, the second factor is sin(n pi y / L), and
    the sines take corner-based coordinates x + L/2, y + L/2. The series is
    truncated at m, n <= kmax (kmax = 99 gives 50 odd terms per index).
    Separable form: P = sum_m sum_n C_mn sin(m pi xs/L) sin(n pi ys/L).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ks = np.arange(1, kmax + 1, 2, dtype=np.float64)  # odd 1..kmax
    mm, nn = np.meshgrid(ks, ks, indexing="ij")
    coef = -32.0 * omega * omega / (mm * nn * np.pi ** 2 *
                                    ((mm * np.pi / L) ** 2 + (nn * np.pi / L) ** 2))
    out = np.empty(x.shape[0])

    def rows(a: int, b: int) -> None:
        xs = (x[a:b] + 0.5 * L) / L
        ys = (y[a:b] + 0.5 * L) / L
        sx = np.sin(np.pi * np.outer(xs, ks))  # (rows, K)
        sy = np.sin(np.pi * np.outer(ys, ks))
        # P_i = sum_mn sx[i,m] coef[m,n] sy[i,n]
        out[a:b] = rho * np.sum((sx @ coef) * sy, axis=1)

    # Fixed row chunks bound the (N, K) temporaries; chunks are independent,
    # so the result does not depend on how many threads evaluate them.
    chunk = 1 << 20
    spans = [(a, min(a + chunk, x.shape[0])) for a in range(0, x.shape[0], chunk)]
    if len(spans) <= 1:
        for a, b in spans:
            rows(a, b)
    else:
        import os
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(lambda ab: rows(*ab), spans))
    return out


def square_patch(n_side: int = 20, nz: int | None = None, L: float = 1.0,
                 omega: float = 5.0, rho0: float = 1.0, h_factor: float = 1.5,
                 jitter: float = 0.01, seed: int = 0, with_pressure: bool = True,
                 kmax: int = 99) -> SphIC:
    """Rotating square patch, 3D extrusion periodic in z (Sec. 5.1).

    Lattice spacing d = L / n_side, nodes at (i + 1/2) d - L/2 in x and y (so
    the rotation is about the square's centre) and (k + 1/2) d in z, with
    Lz = nz * d. id = (i * n_side + j) * nz + k. Each coordinate is displaced
    by d * U(-jitter, +jitter) drawn as one (N, 3) array from
    numpy.random.default_rng(seed). The velocity is set from the displaced
    x, y. h = h_factor * d, m = rho0 d^3, u = 0, c0 = 10 omega L.
    """
    nz = n_side if nz is None else nz
    d = L / n_side
    i, j, k = np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(nz),
                          indexing="ij")
    i = i.ravel().astype(np.float64)
    j = j.ravel().astype(np.float64)
    k = k.ravel().astype(np.float64)
    n = i.size
    x = (i + 0.5) * d - 0.5 * L
    y = (j + 0.5) * d - 0.5 * L
    z = (k + 0.5) * d
    if jitter:
        rng = np.random.default_rng(seed)
        J = rng.uniform(-jitter, jitter, size=(n, 3)) * d
        x = x + J[:, 0]
        y = y + J[:, 1]
        z = z + J[:, 2]
    vx = omega * y
    vy = -omega * x
    vz = np.zeros(n)
    h = np.full(n, h_factor * d)
    m = np.full(n, rho0 * d ** 3)
    u = np.zeros(n)
    if with_pressure:
        p_bg = square_patch_pressure(x, y, L=L, omega=omega, rho=rho0, kmax=kmax)
    else:
        p_bg = np.zeros(n)
    pid = np.arange(n, dtype=np.int32)
    lz = nz * d
    margin = 4.0 * h_factor * d
    lo = (-0.5 * L - margin, -0.5 * L - margin, 0.0)
    hi = (0.5 * L + margin, 0.5 * L + margin, lz)
    params = SphParams(eos=0, rho0=rho0, c0=10.0 * omega * L)
    return SphIC(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, u=u, h=h, m=m, p_bg=p_bg,
                 id=pid, lo=lo, hi=hi, periodic=(0, 0, 1), params=params,
                 meta=dict(kind="square_patch", n_side=n_side, nz=nz, L=L,
                           omega=omega, spacing=d, seed=seed, jitter=jitter))


def lattice_periodic(n_side: int = 16, spacing: float = 2.0 ** -4,
                     h_factor: float = 1.5, rho0: float = 1.0,
                     jitter: float = 0.0, seed: int = 0) -> SphIC:
    """Fully periodic cubic lattice at rest (nodes at (i + 1/2) * spacing).

    With spacing a power of two every coordinate difference and r^2 is exact
    in binary, which makes the on-shell pairs at r = 2h land exactly on the
    cut.
    """
    d = spacing
    i, j, k = np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side),
                          indexing="ij")
    x = (i.ravel() + 0.5) * d
    y = (j.ravel() + 0.5) * d
    z = (k.ravel() + 0.5) * d
    n = x.size
    if jitter:
        rng = np.random.default_rng(seed)
        J = rng.uniform(-jitter, jitter, size=(n, 3)) * d
        x, y, z = x + J[:, 0], y + J[:, 1], z + J[:, 2]
    zero = np.zeros(n)
    L = n_side * d
    return SphIC(x=x.astype(np.float64), y=y.astype(np.float64),
                 z=z.astype(np.float64), vx=zero.copy(), vy=zero.copy(),
                 vz=zero.copy(), u=zero.copy(), h=np.full(n, h_factor * d),
                 m=np.full(n, rho0 * d ** 3), p_bg=zero.copy(),
                 id=np.arange(n, dtype=np.int32), lo=(0.0, 0.0, 0.0),
                 hi=(L, L, L), periodic=(1, 1, 1),
                 params=SphParams(eos=0, rho0=rho0, c0=10.0),
                 meta=dict(kind="lattice", n_side=n_side, spacing=d))


def random_cloud(n: int, seed: int = 0, box: float = 1.0, h_min: float = 0.03,
                 h_max: float = 0.03, periodic=(0, 0, 0),
                 velocity: float = 1.0) -> SphIC:
    """Uniform random cloud in [0, box)^3 with h ~ U[h_min, h_max]."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, box, size=(n, 3))
    V = rng.uniform(-velocity, velocity, size=(n, 3))
    h = rng.uniform(h_min, h_max, size=n) if h_max > h_min else np.full(n, h_min)
    u = rng.uniform(0.5, 1.5, size=n)
    m = rng.uniform(0.5, 1.5, size=n) / n
    pb = rng.uniform(-0.1, 0.1, size=n)
    return SphIC(x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(),
                 vx=V[:, 0].copy(), vy=V[:, 1].copy(), vz=V[:, 2].copy(),
                 u=u, h=h, m=m, p_bg=pb, id=np.arange(n, dtype=np.int32),
                 lo=(0.0, 0.0, 0.0), hi=(box, box, box),
                 periodic=tuple(int(p) for p in periodic),
                 params=SphParams(eos=1, rho0=1.0, c0=1.0),
                 meta=dict(kind="cloud", seed=seed))


def evrard(n: int = 100_000, seed: int = 0, R: float = 1.0, M: float = 1.0,
           u0: float = 0.05, n_target: float = 100.0) -> SphIC:
    """Evrard sphere sample (Sec. 5.1, Evrard profile rho = M / (2 pi R^2 r)).

    M(<r) = M (r/R)^2, so the radius is sampled as r = R sqrt(U1); the
    direction is isotropic (cos(theta) = 2 U2 - 1, phi = 2 pi U3). Equal
    masses M/n, u = u0, v = 0. The smoothing length is the analytic first
    guess for ~n_target gather neighbours under that profile,
    2h = (1.5 n_target R^2 r / n)^(1/3); refining it by neighbour counting is
    a step of the method, not of the input.
    """
    rng = np.random.default_rng(seed)
    U = rng.random((n, 3))
    r = R * np.sqrt(U[:, 0])
    ct = 2.0 * U[:, 1] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * U[:, 2]
    x = r * st * np.cos(ph)
    y = r * st * np.sin(ph)
    z = r * ct
    h = 0.5 * np.cbrt(1.5 * n_target * R * R * r / n)
    # keep the innermost guesses finite and not absurdly small
    h = np.maximum(h, 0.5 * np.cbrt(1.5 * n_target * R * R * (R / n) / n))
    zero = np.zeros(n)
    ext = R * 1.05
    return SphIC(x=x, y=y, z=z, vx=zero.copy(), vy=zero.copy(), vz=zero.copy(),
                 u=np.full(n, u0), h=h, m=np.full(n, M / n), p_bg=zero.copy(),
                 id=np.arange(n, dtype=np.int32), lo=(-ext, -ext, -ext),
                 hi=(ext, ext, ext), periodic=(0, 0, 0),
                 params=SphParams(eos=1, rho0=1.0, c0=1.0, gamma_gas=5.0 / 3.0),
                 meta=dict(kind="evrard", seed=seed, R=R, M=M, u0=u0))
