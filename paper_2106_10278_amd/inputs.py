"""Seeded synthetic catalogues for the NPCF estimator.

This module holds no arithmetic of the estimator itself: it only draws point
sets and weights.  Both the GPU path and the FP64 CPU oracle consume its
output.

Every coordinate is placed on the lattice box * q / 2^32 (q an unsigned
32-bit integer per axis), so that the double-precision positions are exact
and a fixed-point copy of them loses nothing.

The workloads stand in for the data the paper discusses (galaxy surveys,
turbulence simulations); none of those data sets is used.  Recipes:

* ``uniform``    -- n points uniform in a periodic box.
* ``clustered``  -- Poisson-sampled Gaussian blobs: ``n_blob`` points, each
  picks one of ``n_centres`` uniform centres and is offset by N(0, sigma^2) per
  axis (wrapped), plus ``n_uniform`` uniform background points.
* the isotropic 5PCF workload uses ``uniform`` in a unit cube, as the
  paper's 5PCF timing test does.
* ``lognormal_grid`` -- a field on a periodic grid (the gridded-data
  estimator's input): a Gaussian random field with power spectrum
  P(k) ~ k^slope (random phases, unit variance), mapped to a log-normal
  contrast X = exp(sigma g - sigma^2 / 2) - 1, as a stand-in for the density
  of a turbulence simulation.
* ``sphere_points`` / ``s3_points`` -- n points uniform on the unit 2- or
  3-sphere (normalised Gaussian vectors); ``clustered_sphere`` -- Gaussian
  blobs projected onto the sphere plus a uniform background.
* ``hyperbolic_ball`` / ``hyperbolic_clustered`` -- points of hyperbolic space
  H^D on the hyperboloid x0^2 - |x|^2 = 1: uniform in a geodesic ball about
  the origin (radius by inverse transform of the tabulated radial law
  sinh^{D-1} r), and Gaussian blobs of tangent vectors at ball-uniform
  centres carried there by the boost that moves the origin to the centre.
* ``vorticity_tracers`` (D = 2) -- points drawn with density proportional to
  exp(omega) for a random-phase field omega on a grid, whose per-mode
  amplitude falls as 1/|k| (shell energy spectrum ~ k^-3), normalised to
  unit variance.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO32 = float(2 ** 32)


def to_lattice(x: np.ndarray, box) -> np.ndarray:
    """Snap coordinates [D][n] onto the box * q / 2^32 lattice (periodic)."""
    box = np.asarray(box, dtype=np.float64).reshape(-1, 1)
    q = np.floor(np.mod(x, box) / box * TWO32)
    q = np.mod(q, TWO32)
    return q * box / TWO32


def uniform(rng: np.random.Generator, n: int, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    x = rng.uniform(0.0, 1.0, size=(len(box), n)) * box[:, None]
    return to_lattice(x, box)


def clustered(rng: np.random.Generator, n_blob: int, n_uniform: int, n_centres: int, sigma: float, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    D = len(box)
    centres = rng.uniform(0.0, 1.0, size=(D, n_centres)) * box[:, None]
    pick = rng.integers(0, n_centres, size=n_blob)
    blob = centres[:, pick] + rng.normal(0.0, sigma, size=(D, n_blob))
    back = rng.uniform(0.0, 1.0, size=(D, n_uniform)) * box[:, None]
    return to_lattice(np.concatenate([blob, back], axis=1), box)


def vorticity_tracers(rng: np.random.Generator, n: int, grid: int, box: float) -> np.ndarray:
    white = rng.normal(size=(grid, grid))
    fk = np.fft.rfft2(white)
    kx = np.fft.fftfreq(grid) * grid
    ky = np.fft.rfftfreq(grid) * grid
    kk = np.sqrt(kx[:, None] ** 2 + ky[None, :] ** 2)
    filt = np.zeros_like(kk)
    band = (kk >= 1.0) & (kk <= grid // 2)
    filt[band] = 1.0 / kk[band]
    omega = np.fft.irfft2(fk * filt, s=(grid, grid))
    omega = (omega - omega.mean()) / omega.std()
    dens = np.exp(omega).ravel()
    cdf = np.cumsum(dens)
    cdf /= cdf[-1]
    cell = np.searchsorted(cdf, rng.uniform(0.0, 1.0, size=n), side="right")
    cell = np.minimum(cell, grid * grid - 1)
    ix, iy = np.divmod(cell, grid)
    h = box / grid
    x = (ix + rng.uniform(0.0, 1.0, size=n)) * h
    y = (iy + rng.uniform(0.0, 1.0, size=n)) * h
    return to_lattice(np.stack([x, y]), [box, box])


def lognormal_grid(rng: np.random.Generator, dims, slope: float = -11.0 / 3.0, sigma: float = 1.0) -> np.ndarray:
    dims = tuple(int(d) for d in dims)
    white = rng.normal(size=dims)
    fk = np.fft.rfftn(white)
    ks = np.meshgrid(*[np.fft.fftfreq(d) * d for d in dims[:-1]], np.fft.rfftfreq(dims[-1]) * dims[-1], indexing="ij")
    kk = np.sqrt(sum(k * k for k in ks))
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (slope / 2.0)
    g = np.fft.irfftn(fk * amp, s=dims, axes=tuple(range(len(dims))))
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g - 0.5 * sigma * sigma) - 1.0


def grid_nodes(dims, box) -> np.ndarray:
    """Node coordinates [D][prod dims] of a periodic grid (row-major, last axis
    fastest), node (i_0, ..) at x_k = i_k box_k / dims_k."""
    axes = [np.arange(d) * (b / d) for d, b in zip(dims, box)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return to_lattice(np.stack([m.ravel() for m in mesh]), box)


@dataclasses.dataclass
class Workload:
    name: str
    D: int
    N: int
    lmax: int
    edges: np.ndarray
    box: list
    pos: np.ndarray          # [D][n] float64 on the lattice
    w: np.ndarray            # [n] float64
    n_data: int = 0          # leading points that are data (rest: randoms)
    note: str = ""
    Lmax: object = None      # line-of-sight basis (D = 3, N = 3): largest L; None: isotropic
    field: object = None     # gridded data: the field on the grid (pos and w are then its nodes)
    sphere: bool = False     # points on the unit D-sphere: pos [D + 1][n] unit vectors, edges in radians
    hyperbolic: bool = False  # points of H^D on the hyperboloid: pos [D + 1][n], box[0] = the region's volume


def c1_small_3pcf(seed: int = 1001) -> Workload:
    """D=3, N=3: 2000 uniform points, periodic cube of side 100, w = 1,
    8 linear bins in [2, 20], lmax = 4."""
    rng = np.random.default_rng(seed)
    box = [100.0] * 3
    pos = uniform(rng, 2000, box)
    return Workload("D3-N3-uniform-2k", 3, 3, 4, np.linspace(2.0, 20.0, 9), box, pos, np.ones(2000), 2000)


def c2_clustered_4pcf(seed: int = 1002, n_data: int = 200_000, n_rand: int = 600_000) -> Workload:
    """D=3, N=4: 200k clustered data (half in 2000 Gaussian blobs of sigma 5,
    half uniform), w = +1, plus 600k uniform randoms with w = -1/3, periodic
    cube of side 1000, 10 linear bins in [20, 160], lmax = 5."""
    rng = np.random.default_rng(seed)
    box = [1000.0] * 3
    data = clustered(rng, n_data // 2, n_data - n_data // 2, 2000, 5.0, box)
    rand = uniform(rng, n_rand, box)
    pos = np.concatenate([data, rand], axis=1)
    w = np.concatenate([np.ones(n_data), np.full(n_rand, -1.0 / 3.0)])
    return Workload(f"D3-N4-clustered-{n_data // 1000}k+{n_rand // 1000}k-randoms", 3, 4, 5,
                    np.linspace(20.0, 160.0, 11), box, pos, w, n_data)


def c6_los_3pcf(seed: int = 1006, n_data: int = 200_000, n_rand: int = 600_000) -> Workload:
    """D=3, N=3, line-of-sight basis (L <= 6): the shape of the clustered
    800k-point catalogue (c2_clustered_4pcf) with redshift-space-like
    anisotropy -- blob offsets along axis 3 four times wider (sigma 20 against
    5 across) -- 200k data (half in 2000 blobs, half uniform), w = +1, plus
    600k uniform randoms with w = -1/3, periodic cube of side 1000, 10 linear
    bins in [20, 160], lmax = 5."""
    rng = np.random.default_rng(seed)
    box = np.array([1000.0] * 3)
    nb = n_data // 2
    centres = rng.uniform(0.0, 1.0, size=(3, 2000)) * box[:, None]
    pick = rng.integers(0, 2000, size=nb)
    sig = np.array([5.0, 5.0, 20.0])[:, None]
    blob = centres[:, pick] + rng.normal(0.0, 1.0, size=(3, nb)) * sig
    back = rng.uniform(0.0, 1.0, size=(3, n_data - nb)) * box[:, None]
    rand = rng.uniform(0.0, 1.0, size=(3, n_rand)) * box[:, None]
    pos = to_lattice(np.concatenate([blob, back, rand], axis=1), box)
    w = np.concatenate([np.ones(n_data), np.full(n_rand, -1.0 / 3.0)])
    return Workload(f"D3-N3-los-Lmax6-rsd-{n_data // 1000}k+{n_rand // 1000}k-randoms", 3, 3, 5,
                    np.linspace(20.0, 160.0, 11), list(box), pos, w, n_data, Lmax=6)


def c7_uniform_5pcf(seed: int = 1007, n: int = 100_000) -> Workload:
    """D=3, N=5 (isotropic 5PCF): n uniform points in a periodic unit cube,
    w = 1, 10 linear bins in [0.1, 0.4], lmax = 4 -- the setting of the paper's
    5PCF timing test (section "Hydrodynamic Turbulence"), at a fixed n."""
    rng = np.random.default_rng(seed)
    box = [1.0] * 3
    pos = uniform(rng, n, box)
    return Workload(f"D3-N5-uniform-{n // 1000}k", 3, 5, 4, np.linspace(0.1, 0.4, 11), box, pos, np.ones(n), n)


def grid_workload(name: str, D: int, N: int, lmax: int, dims, box, edges, seed: int, sigma: float = 1.0) -> Workload:
    """A gridded-data workload: the log-normal field on the grid, and its node
    catalogue (positions, weights X dV) for the pair path and the oracle."""
    rng = np.random.default_rng(seed)
    field = lognormal_grid(rng, dims, sigma=sigma)
    pos = grid_nodes(dims, box)
    dV = float(np.prod([b / d for d, b in zip(dims, box)]))
    n = pos.shape[1]
    return Workload(name, D, N, lmax, np.asarray(edges, dtype=np.float64), list(box), pos, field.ravel() * dV, n,
                    field=field)


def c8_grid_4pcf(seed: int = 1008, g: int = 128) -> Workload:
    """D=3, N=4 on gridded data: a log-normal field (spectrum k^-11/3, sigma 1)
    on a periodic 128^3 grid of unit spacing, 10 linear bins in [2, 12],
    lmax = 4 (section "Application to Gridded Data")."""
    return grid_workload(f"D3-N4-grid-{g}^3-lognormal", 3, 4, 4, (g, g, g), [float(g)] * 3, np.linspace(2.0, 12.0, 11),
                         seed)


def c3_vorticity_4pcf(seed: int = 1003, n: int = 500_000, grid: int = 1024) -> Workload:
    """D=2, N=4: tracers of exp(vorticity) on a periodic square of side 2 pi,
    w = 1, 12 linear bins in [0.02, 0.5], |l| <= 8."""
    rng = np.random.default_rng(seed)
    box = 2.0 * math.pi
    pos = vorticity_tracers(rng, n, grid, box)
    return Workload(f"D2-N4-vorticity-{n // 1000}k", 2, 4, 8, np.linspace(0.02, 0.5, 13), [box, box], pos, np.ones(n), n)


def c4_batch_sizes(count: int = 64, seed: int = 4000) -> list:
    """Data sizes of the batched workload: log-uniform in [20k, 300k]."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(20_000), math.log(300_000))))) for _ in range(count)]


def c4_catalogue(c: int, n_data: int) -> Workload:
    """One catalogue of the batched D=3, N=4 workload (seed 4000 + c): the
    clustered generator (c2_clustered_4pcf) plus 3 n_data uniform randoms at w = -1/3."""
    return c2_clustered_4pcf(seed=4000 + c, n_data=n_data, n_rand=3 * n_data)


def c5_hyper_3pcf(seed: int = 1005, n_blob: int = 1_000_000, n_uniform: int = 1_000_000) -> Workload:
    """D=4, N=3: 2M points (1M in 2000 Gaussian blobs of sigma 5, 1M uniform)
    in a periodic hypercube of side 500, w ~ N(1, 0.1^2), 10 linear bins in
    [5, 50], lmax = 6."""
    rng = np.random.default_rng(seed)
    box = [500.0] * 4
    pos = clustered(rng, n_blob, n_uniform, 2000, 5.0, box)
    n = pos.shape[1]
    w = rng.normal(1.0, 0.1, size=n)
    return Workload(f"D4-N3-clustered-{n // 1000}k", 4, 3, 6, np.linspace(5.0, 50.0, 11), box, pos, w, n)


def tiny(D: int, N: int, lmax: int, n: int, seed: int, box_side: float = 10.0, rmax: float = 4.0,
         nbins: int = 3, weights: str = "mixed") -> Workload:
    """Small periodic catalogue for brute-force and parity tests."""
    rng = np.random.default_rng(seed)
    box = [box_side] * D
    pos = uniform(rng, n, box)
    if weights == "ones":
        w = np.ones(n)
    else:
        w = rng.uniform(-0.5, 1.5, size=n)
    edges = np.linspace(rmax / (nbins + 1), rmax, nbins + 1)
    return Workload(f"tiny-D{D}-N{N}-{n}", D, N, lmax, edges, box, pos, w, n)


def sphere_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """n points uniform on the unit 2-sphere: unit vectors [3][n] (normalised
    Gaussian triples)."""
    x = rng.normal(size=(3, n))
    return x / np.linalg.norm(x, axis=0)


def c9_sphere_4pcf(seed: int = 1009, n: int = 100_000) -> Workload:
    """D=2, N=4 on the unit 2-sphere: n uniform points, w = 1, 10 bins equal
    in cos(theta) over [-0.5, 0.5) (great-circle angles 60 to 120 degrees),
    lmax = 4 -- the paper's CMB timing test (35 angular, 120 radial
    components), at a fixed n."""
    rng = np.random.default_rng(seed)
    pos = sphere_points(rng, n)
    edges = np.arccos(np.linspace(0.5, -0.5, 11))
    return Workload(f"S2-N4-uniform-{n // 1000}k", 2, 4, 4, edges, [1.0, 1.0], pos, np.ones(n), n, sphere=True)


def s3_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """n points uniform on the unit 3-sphere: unit vectors [4][n] (normalised
    Gaussian quadruples)."""
    x = rng.normal(size=(4, n))
    return x / np.linalg.norm(x, axis=0)


def clustered_sphere(rng: np.random.Generator, D: int, n_blob: int, n_uniform: int, n_centres: int,
                     sigma: float) -> np.ndarray:
    """Points on the unit D-sphere [D + 1][n]: ``n_blob`` points, each a
    uniform centre (one of ``n_centres``) offset by N(0, sigma^2) per
    coordinate of R^{D+1} and projected back onto the sphere (blobs of
    angular size about sigma), then ``n_uniform`` uniform points."""
    c = s3_points(rng, n_centres) if D == 3 else sphere_points(rng, n_centres)
    pick = rng.integers(0, n_centres, size=n_blob)
    x = c[:, pick] + rng.normal(0.0, sigma, size=(D + 1, n_blob))
    x /= np.linalg.norm(x, axis=0)
    back = s3_points(rng, n_uniform) if D == 3 else sphere_points(rng, n_uniform)
    return np.concatenate([x, back], axis=1)


def c10_s3_4pcf(seed: int = 1010, n_blob: int = 90_000, n_uniform: int = 10_000) -> Workload:
    """D=3, N=4 on the unit 3-sphere (curvature k = 1): 100k points, 90k in
    50 blobs of angular size 0.2 rad and 10k uniform, w = 1, 10 bins equal in
    geodesic angle over [pi/6, pi/2], lmax = 5 (the 111 components of the flat
    D=3 4PCF workload).  The paper gives the constant-curvature estimator
    without a timing test; this stands in for one, with bins as wide as the
    sky test's and structure on the scale of the bins."""
    rng = np.random.default_rng(seed)
    pos = clustered_sphere(rng, 3, n_blob, n_uniform, 50, 0.2)
    n = pos.shape[1]
    edges = np.linspace(math.pi / 6, math.pi / 2, 11)
    return Workload(f"S3-N4-clustered-{n // 1000}k", 3, 4, 5, edges, [1.0, 1.0, 1.0], pos, np.ones(n), n, sphere=True)


def hyperbolic_ball(rng: np.random.Generator, D: int, n: int, R: float) -> np.ndarray:
    """n points uniform (in the volume element sinh^{D-1} r dr dOmega) in the
    geodesic ball of radius R about the origin of H^D: [D + 1][n] hyperboloid
    coordinates (cosh r, sinh r * direction)."""
    grid = np.linspace(0.0, R, 4097)
    dens = np.sinh(grid) ** (D - 1)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    r = np.interp(rng.uniform(0.0, cdf[-1], size=n), cdf, grid)
    d = rng.normal(size=(D, n))
    d /= np.linalg.norm(d, axis=0)
    return np.vstack([np.cosh(r), np.sinh(r) * d])


def _boost_to(c: np.ndarray) -> np.ndarray:
    """The Lorentz boost of R^{D,1} that takes the origin (1, 0, .., 0) to the
    hyperboloid point c."""
    D = len(c) - 1
    B = np.eye(D + 1)
    B[0, 0] = c[0]
    B[0, 1:] = B[1:, 0] = c[1:]
    B[1:, 1:] += np.outer(c[1:], c[1:]) / (1.0 + c[0])
    return B


def hyperbolic_clustered(rng: np.random.Generator, D: int, n_blob: int, n_uniform: int, n_centres: int,
                         sigma: float, R: float) -> np.ndarray:
    """Points of H^D: ``n_blob`` in blobs (a ball-uniform centre, one of
    ``n_centres``, and a tangent vector with N(0, sigma^2) coordinates taken
    along the geodesics from the centre), then ``n_uniform`` ball-uniform
    points (radius R)."""
    centres = hyperbolic_ball(rng, D, n_centres, R)
    pick = rng.integers(0, n_centres, size=n_blob)
    t = rng.normal(0.0, sigma, size=(D, n_blob))
    r = np.linalg.norm(t, axis=0)
    local = np.vstack([np.cosh(r), np.sinh(r) * t / r])
    blob = np.empty_like(local)
    for c in range(n_centres):
        sel = pick == c
        blob[:, sel] = _boost_to(centres[:, c]) @ local[:, sel]
    return np.concatenate([blob, hyperbolic_ball(rng, D, n_uniform, R)], axis=1)


def c11_h3_4pcf(seed: int = 1011, n_blob: int = 80_000, n_uniform: int = 20_000) -> Workload:
    """D=3, N=4 in hyperbolic space H^3 (curvature k = -1): 100k points, 80k in
    40 blobs of 0.15 and 20k uniform in the geodesic ball of radius 1.5, w = 1,
    10 bins equal in geodesic distance over [0.1, 0.9], lmax = 5; V = the
    ball's volume pi (sinh 3 - 3).  Defined here: the paper gives the
    constant-curvature estimator without a workload on it."""
    rng = np.random.default_rng(seed)
    R = 1.5
    pos = hyperbolic_clustered(rng, 3, n_blob, n_uniform, 40, 0.15, R)
    n = pos.shape[1]
    V = math.pi * (math.sinh(2 * R) - 2 * R)
    edges = np.linspace(0.1, 0.9, 11)
    return Workload(f"H3-N4-clustered-{n // 1000}k", 3, 4, 5, edges, [V, 1.0, 1.0], pos, np.ones(n), n,
                    hyperbolic=True)
