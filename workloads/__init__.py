"""Seeded synthetic inputs for the 2D FDFD solves: permittivity maps and sources.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the solver method itself: it only draws permittivity maps
(grating-shaped structures and optimisation-trajectory-like sequences of them)
and builds the right-hand side b = -i*omega*J of the frequency-domain Maxwell
equation (Sec. 2, Eq. 1) from a current density J.

The paper's own data set (about 30,000 optimised grating splitters, Methods)
is not public; these generators stand in for it with the same kind of
structure: a silicon (eps 12.25) waveguide on silica (eps 2.085), a design
region whose permittivity is continuous between the two, 20-25 nm cells and
10^4-10^5 unknowns, and sequences of correlated permittivities as produced by
the steps of a gradient-based design run.

Units: c = mu0 = eps0 = 1, lengths in micrometres, omega = 2*pi/lambda.
Grid layout: row-major with x fastest, flat index = iy*nx + ix.
Every permittivity is returned as float32 so that a single-precision and a
double-precision consumer see exactly the same values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.ndimage import gaussian_filter

EPS_SIO2 = 2.085
EPS_SI = 12.25
CONTRAST = EPS_SI - EPS_SIO2  # 10.165


@dataclasses.dataclass
class Instance:
    """One FDFD problem: A(eps, omega, dx, npml) f = b."""
    eps: np.ndarray          # float32 [ny, nx] relative permittivity
    b: np.ndarray            # complex128 [ny*nx] right-hand side, -i*omega*J
    nx: int
    ny: int
    dx: float                # cell size, um
    wavelength: float        # um
    npml: int                # PML thickness in cells (same on all four sides)
    name: str = ""

    @property
    def omega(self) -> float:
        return 2.0 * math.pi / self.wavelength

    @property
    def D(self) -> int:
        return self.nx * self.ny


def rhs_from_current(J: np.ndarray, omega: float) -> np.ndarray:
    """b = -i omega J (right-hand side of Eq. 1 with mu0 = 1), flattened."""
    return (-1j * omega * np.asarray(J, dtype=np.complex128)).reshape(-1)


# ---------------------------------------------------------------------------
# Small binary-pixel problem (64x64 grid, line current)
# ---------------------------------------------------------------------------

def small_binary(seed: int = 0, n: int = 64, dx: float = 0.040,
                 wavelength: float = 1.55, npml: int = 10,
                 lo: int = 16, hi: int = 48, src_ix: int = 12) -> Instance:
    """64x64 grid, silica background, rows/cols [16, 48) random binary pixels
    {2.085, 12.25} (Bernoulli 0.5), unit line current on column ix = 12 (all rows)."""
    rng = np.random.default_rng(seed)
    eps = np.full((n, n), EPS_SIO2)
    pix = rng.random((hi - lo, hi - lo)) < 0.5
    eps[lo:hi, lo:hi] = np.where(pix, EPS_SI, EPS_SIO2)
    eps = eps.astype(np.float32)
    J = np.zeros((n, n))
    J[:, src_ix] = 1.0
    omega = 2 * math.pi / wavelength
    return Instance(eps, rhs_from_current(J, omega), n, n, dx, wavelength, npml,
                    name=f"binary{n}x{n}_s{seed}")


# ---------------------------------------------------------------------------
# Grating-shaped problems
# ---------------------------------------------------------------------------

def design_box(nx: int, ny: int):
    """(x0, y0, wx, wy) of the centred design region: round(5nx/12) x ny/3."""
    wx = int(round(5 * nx / 12))
    wy = ny // 3
    return (nx - wx) // 2, (ny - wy) // 2, wx, wy


def waveguide_rows(ny: int, dx: float, width_um: float = 0.400):
    h = int(round(width_um / dx))
    return ny // 2 - h // 2, ny // 2 - h // 2 + h


def smooth_field(rng: np.random.Generator, shape, sigma: float = 3.0) -> np.ndarray:
    z = rng.standard_normal(shape)
    return gaussian_filter(z, sigma, mode="reflect")


def design_region_eps(seed: int, wx: int, wy: int, sigma: float = 3.0) -> np.ndarray:
    """Continuous design: standardised smoothed Gaussian field through a sigmoid."""
    z = smooth_field(np.random.default_rng(seed), (wy, wx), sigma)
    z = (z - z.mean()) / z.std()
    rho = 1.0 / (1.0 + np.exp(-2.0 * z))
    return EPS_SIO2 + CONTRAST * rho


def grating_eps(region: np.ndarray, nx: int, ny: int, dx: float) -> np.ndarray:
    """Silica background, a 400 nm silicon waveguide through the centre row band
    on both sides of the design region, and the design region itself."""
    x0, y0, wx, wy = design_box(nx, ny)
    eps = np.full((ny, nx), EPS_SIO2)
    r0, r1 = waveguide_rows(ny, dx)
    eps[r0:r1, :x0] = EPS_SI
    eps[r0:r1, x0 + wx:] = EPS_SI
    eps[y0:y0 + wy, x0:x0 + wx] = region
    return eps.astype(np.float32)


def slab_mode_source(eps: np.ndarray, ix: int, dx: float, omega: float) -> np.ndarray:
    """Current density J: the fundamental mode of the column eps[:, ix] placed on
    that column, peak-normalised to +1.

    The mode is the eigenvector with the largest eigenvalue of the real symmetric
    1D operator u -> u'' + omega^2 eps(y) u (second difference, zero outside the
    column ends); this is input construction, not part of the solver.
    """
    ny, nx = eps.shape
    col = eps[:, ix].astype(np.float64)
    L = (np.diag(np.full(ny, -2.0)) + np.diag(np.ones(ny - 1), 1)
         + np.diag(np.ones(ny - 1), -1)) / dx ** 2 + np.diag(omega ** 2 * col)
    w, v = np.linalg.eigh(L)
    u = v[:, -1]
    u = u / u[np.argmax(np.abs(u))]
    J = np.zeros((ny, nx))
    J[:, ix] = u
    return J


def grating(seed: int, nx: int = 480, ny: int = 240, dx: float = 0.025,
            wavelength: float = 1.30, npml: int = 20, region=None,
            name: str | None = None) -> Instance:
    """Grating-shaped instance; the mode source sits at ix = npml + 10."""
    x0, y0, wx, wy = design_box(nx, ny)
    if region is None:
        region = design_region_eps(seed, wx, wy)
    eps = grating_eps(region, nx, ny, dx)
    omega = 2 * math.pi / wavelength
    J = slab_mode_source(eps, npml + 10, dx, omega)
    return Instance(eps, rhs_from_current(J, omega), nx, ny, dx, wavelength, npml,
                    name=name or f"grating{nx}x{ny}_s{seed}")


def perturb_region(region: np.ndarray, seed: int, amp: float = 0.05) -> np.ndarray:
    """One synthetic design step: add amp*contrast times a smoothed normal field
    scaled to max |p| = 1, then clip to [eps_SiO2, eps_Si]."""
    p = smooth_field(np.random.default_rng(seed), region.shape)
    p = p / np.abs(p).max()
    return np.clip(region + amp * CONTRAST * p, EPS_SIO2, EPS_SI)


def trajectory(base_seed: int, step_seed0: int, steps: int, nx: int, ny: int,
               wavelength: float, dx: float = 0.025, npml: int = 20):
    """A synthetic optimisation trajectory: step 0 is a fresh grating design,
    every later step perturbs the previous design region."""
    x0, y0, wx, wy = design_box(nx, ny)
    region = design_region_eps(base_seed, wx, wy)
    out = []
    for s in range(steps):
        if s > 0:
            region = perturb_region(region, step_seed0 + s)
        out.append(grating(base_seed, nx, ny, dx, wavelength, npml, region=region,
                           name=f"traj{base_seed}_step{s}_{nx}x{ny}"))
    return out


BATCH_GRIDS = [(192, 96), (320, 160), (480, 240)]
BATCH_WAVELENGTHS = [1.30, 1.55]


def correlated_batch(n_traj: int = 8, steps: int = 32):
    """n_traj trajectories x steps correlated problems of uneven sizes:
    trajectory t uses grid BATCH_GRIDS[t % 3] and wavelength
    BATCH_WAVELENGTHS[t % 2]; seeds 3000+t (design) and 3000+100t+s (steps)."""
    out = []
    for t in range(n_traj):
        nx, ny = BATCH_GRIDS[t % 3]
        lam = BATCH_WAVELENGTHS[t % 2]
        out.extend(trajectory(3000 + t, 3000 + 100 * t, steps, nx, ny, lam))
    return out


def trajectory_dataset(n_traj: int, steps: int, seed0: int = 70_000, nx: int = 480,
                       ny: int = 240, wavelength: float = 1.30):
    """Synthetic design-trajectory data set: n_traj trajectories of `steps`
    correlated grating designs each (trajectory t: seeds seed0 + t and
    10*seed0 + 100 t + s)."""
    out = []
    for t in range(n_traj):
        out.extend(trajectory(seed0 + t, 10 * seed0 + 100 * t, steps, nx, ny, wavelength))
    return out


def split_train_test(n: int, train_frac: float = 0.75, seed: int = 0):
    """Random split of n examples into training and evaluation index lists
    (the paper's data set is split 75 / 25 over all trajectory steps)."""
    perm = np.random.default_rng(seed).permutation(n)
    ntr = int(round(train_frac * n))
    return sorted(perm[:ntr].tolist()), sorted(perm[ntr:].tolist())


# Named seed ranges for the PCA / CNN workloads (all 480x240, 1.30 um).
PCA_TRAIN_SEED0 = 10_000
PCA_TEST_SEED0 = 20_000
CNN_TRAJ_SEED0 = 40_000
CNN_STEP_SEED0 = 400_000
CNN_TEST_SEED0 = 50_000


def grating_set(seed0: int, count: int, **kw):
    return [grating(seed0 + i, **kw) for i in range(count)]


def cnn_training_trajectories(n_traj: int = 313, steps: int = 32, **kw):
    out = []
    for t in range(n_traj):
        out.append(trajectory(CNN_TRAJ_SEED0 + t, CNN_STEP_SEED0 + 100 * t, steps,
                              kw.get("nx", 480), kw.get("ny", 240),
                              kw.get("wavelength", 1.30)))
    return out


def random_complex(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard complex normal test vectors (for operator and kernel checks)."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
