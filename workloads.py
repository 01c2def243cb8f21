"""Seeded synthetic workload descriptions shared by the oracle and the HIP path.

This module holds *inputs only*: body placements, mesh levels, boundary-condition
flags, wavenumber grids, observation points and pulse parameters.  It contains
none of the method's arithmetic (no mesh construction, no kernels, no spectra),
so that the CPU oracle and the GPU library can both consume it without sharing
any computation.

Lengths are in units of the sphere radius a, the sound speed is c = 1 and the
incident plane wave travels along +z (Sec. IV of the paper: pulse of Eq. (pulse)
travelling in z).  Every random draw comes from ``numpy.random.default_rng``
with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

HARD = 0  # dP/dn prescribed on the surface (sound-hard), P unknown
SOFT = 1  # P prescribed on the surface (sound-soft), dP/dn unknown


@dataclass(frozen=True)
class Body:
    """One scatterer: an icosphere of ``level`` mapped to an ellipsoid.

    The unit icosphere point u maps to center + (radius*u0, radius*u1,
    radius*aspect*u2); aspect > 1 is a prolate spheroid along z.
    """
    center: tuple
    radius: float
    aspect: float
    level: int
    bc: int


@dataclass
class Pulse:
    """Incident waveform in the travelling coordinate s = z - t (c = 1)."""
    kind: str            # 'paper', 'gauss', 'ricker', 'nwave', 'chirp', 'gsine'
    params: dict = field(default_factory=dict)


@dataclass
class Workload:
    name: str
    bodies: List[Body]
    k: np.ndarray                 # wavenumbers, float64, strictly positive
    points: np.ndarray            # observation points [M,3] float64
    pulses: List[Pulse]
    T: int                        # time samples of the synthesis
    dk: float                     # uniform wavenumber spacing of the grid
    z_shift: float                # pulse origin: incident field is F(z - t - z_shift)
    rescale_area: bool = True
    notes: str = ""


def two_sphere_gap(seed: int = 0) -> float:
    """Surface-to-surface gap of the two-sphere configuration, U(0.2, 3.0)."""
    return float(np.random.default_rng(seed).uniform(0.2, 3.0))


def two_spheres(level: int = 4, seed: int = 0, bc: int = HARD) -> List[Body]:
    g = two_sphere_gap(seed)
    h = 1.0 + 0.5 * g
    return [Body((0.0, 0.0, -h), 1.0, 1.0, level, bc),
            Body((0.0, 0.0, h), 1.0, 1.0, level, bc)]


def uniform_k(kmax: float, n: int) -> np.ndarray:
    """k_m = kmax*m/n for m = 1..n (the m = 0 term carries no scattering)."""
    return kmax * np.arange(1, n + 1, dtype=np.float64) / n


def ring_points(radius: float, n: int) -> np.ndarray:
    """n points on a circle of given radius in the xz-plane, theta_i = 2*pi*i/n."""
    th = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    return np.stack([radius * np.sin(th), np.zeros(n), radius * np.cos(th)], axis=1)


def plane_grid(n: int, half: float = 10.0) -> np.ndarray:
    """n*n cell-centred points on the plane x = 0, y,z in [-half, half]."""
    c = -half + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 * half / n)
    yy, zz = np.meshgrid(c, c, indexing="ij")
    return np.stack([np.zeros(n * n), yy.ravel(), zz.ravel()], axis=1)


def sphere_l2_workload() -> Workload:
    """Single sound-hard sphere, level-2 icosphere (162 nodes), 32 k in (0,6]."""
    return Workload(
        name="sphere_L2_hard_32k",
        bodies=[Body((0.0, 0.0, 0.0), 1.0, 1.0, 2, HARD)],
        k=uniform_k(6.0, 32), points=ring_points(2.0, 32),
        pulses=[Pulse("gaussk", {"k0": 3.0, "width": 1.0})],
        T=64, dk=6.0 / 32, z_shift=0.0)


def two_spheres_workload(n_k: int = 512) -> Workload:
    """Two sound-hard spheres (2 x 2562 nodes, N = 5124), k in (0,12]."""
    return Workload(
        name="two_spheres_L4_hard_512k",
        bodies=two_spheres(4, 0, HARD),
        k=uniform_k(12.0, n_k), points=plane_grid(32),
        pulses=[Pulse("gsine", {"k0": 6.0, "sigma": 1.5})],
        T=2 * n_k, dk=12.0 / n_k, z_shift=-12.0)


def uneven_bodies_workload(seed: int = 0, n_k: int = 1024) -> Workload:
    """Eight scatterers of uneven size: radius U(0.3,1.5), sphere or prolate
    spheroid (aspect U(1,3)), level in {3,4,5}, one hard/soft flag each.
    Each body is an independent scattering problem."""
    rng = np.random.default_rng(seed)
    bodies = []
    for _ in range(8):
        radius = float(rng.uniform(0.3, 1.5))
        prolate = bool(rng.integers(0, 2))
        aspect = float(rng.uniform(1.0, 3.0)) if prolate else 1.0
        level = int(rng.integers(3, 6))
        bc = int(rng.integers(0, 2))
        bodies.append(Body((0.0, 0.0, 0.0), radius, aspect, level, bc))
    return Workload(name="uneven_8_bodies", bodies=bodies,
                    k=uniform_k(12.0, n_k), points=np.zeros((0, 3)), pulses=[],
                    T=2 * n_k, dk=12.0 / n_k, z_shift=0.0)


def surrogate_train_k(n: int = 256) -> np.ndarray:
    """Training wavenumbers of the surrogate: cell centres of (0,12]."""
    return 12.0 * (np.arange(1, n + 1, dtype=np.float64) - 0.5) / n


def surrogate_workload() -> Workload:
    return Workload(name="surrogate_two_spheres", bodies=two_spheres(4, 0, HARD),
                    k=uniform_k(12.0, 4096), points=np.zeros((0, 3)), pulses=[],
                    T=8192, dk=12.0 / 4096, z_shift=0.0)


def spacetime_pulses(seed: int = 0) -> List[Pulse]:
    """Four incident pulses with seeded widths: Gaussian, Ricker, N-wave, chirp."""
    out = []
    for q, kind in enumerate(("gauss", "ricker", "nwave", "chirp")):
        rng = np.random.default_rng(seed + q)
        if kind == "chirp":
            out.append(Pulse(kind, {"ka": float(rng.uniform(2.0, 4.0)),
                                    "kb": float(rng.uniform(6.0, 9.0)),
                                    "D": float(rng.uniform(2.0, 4.0))}))
        else:
            out.append(Pulse(kind, {"sigma": float(rng.uniform(0.5, 1.5))}))
    return out


def spacetime_workload(n_grid: int = 1024, n_k: int = 2048) -> Workload:
    return Workload(name="spacetime_two_spheres_1M", bodies=two_spheres(4, 0, HARD),
                    k=uniform_k(12.0, n_k), points=plane_grid(n_grid),
                    pulses=spacetime_pulses(0), T=2 * n_k, dk=12.0 / n_k,
                    z_shift=-12.0)


def paper_sphere_pulse(n_cycles2: int = 4, alpha: float = 0.1, w: float = 20.1):
    """The pulse of the spherical-scatterer results: 2N_c cycles, modulation
    alpha, total width w (Sec. IV A)."""
    return Pulse("paper", {"Nc": n_cycles2 / 2.0, "alpha": alpha, "w": w})


def seeded_complex(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def mlp_initial_weights(sizes, seed: int = 0):
    """Seeded initial weights of the surrogate network, an input shared by the
    GPU trainer and the reference: W_i ~ U(-sqrt(6/in), sqrt(6/in)) [in, out]
    float32, b_i = 0."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        out.append((rng.uniform(-lim, lim, (a, b)).astype(np.float32), np.zeros(b, np.float32)))
    return out


def interior_points(bodies: List[Body], per_body: int = 8, seed: int = 0,
                    frac=(0.2, 0.6)) -> np.ndarray:
    """Random points strictly inside each body (seeded): a direction uniform on
    the sphere and a radius fraction uniform in ``frac`` of the body's
    semi-axes, [len(bodies) * per_body, 3].  Auxiliary collocation points for
    the interior-point conditions that remove fictitious resonances."""
    rng = np.random.default_rng(seed)
    out = []
    for b in bodies:
        v = rng.normal(size=(per_body, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        t = rng.uniform(frac[0], frac[1], size=(per_body, 1))
        u = v * t
        out.append(np.asarray(b.center)[None, :] + u * np.array([b.radius, b.radius, b.radius * b.aspect]))
    return np.concatenate(out).astype(np.float64)


# Interior Dirichlet eigenvalues k a of the unit sphere below 8: zeros of the
# spherical Bessel functions j_0 (pi, 2 pi), j_1, j_2, j_3 (standard tables,
# rounded to 4 decimals).  The surface equation of a sphere is nearly singular
# at these wavenumbers.
SPHERE_RESONANCES = (3.1416, 4.4934, 5.7635, 6.2832, 6.9879, 7.7253)

