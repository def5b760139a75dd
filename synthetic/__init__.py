"""Seeded synthetic inputs for the lattice Boltzmann step.

This module is shared by the HIP path's tests/benchmarks and by the CPU oracle.
It produces only *inputs*: node-type maps, initial macroscopic fields (density,
velocity) and seeded perturbations.  It contains none of the method's
arithmetic (no equilibria, no collision, no streaming).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), evaluated on a counter:
``u = (splitmix64(seed ^ counter) >> 11) * 2**-53``, with
``counter = stream * count + flat_index``.  Both sides receive the drawn
numbers as input arrays, so there is no device RNG to keep in sync.

Workload shapes follow the configurations the method is measured on (see the
paper's benchmark section: duct flows, periodic vortices, two-component
periodic boxes); every shape here is synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DEFAULT_SEED = 20131124

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to uint64 states."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` doubles in [0, 1) for counters ``stream*count_total + start + k``.

    ``start`` lets a caller fill a long stream in chunks; the value at a given
    flat index does not depend on the chunking.
    """
    idx = np.arange(start, start + count, dtype=np.uint64)
    key = np.uint64(seed) ^ (np.uint64(stream) * np.uint64(1 << 40) + idx)
    bits = splitmix64(key) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm(seed: int, stream: int, shape, amp: float, dtype=np.float64) -> np.ndarray:
    """Array of ``shape`` with entries drawn from U(-amp, amp), flat C order."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=dtype)
    chunk = 1 << 24
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        out[s:s + c] = amp * (2.0 * uniform01(seed, stream, c, s) - 1.0)
    return out.reshape(shape)


# ---------------------------------------------------------------------------
# lattice identifiers shared with the C ABI (plain integers, no tables)
D2Q9, D3Q19 = 0, 1
BGK, MRT, ELBM, SHANCHEN, REG, SMAG, FREE_ENERGY = 0, 1, 2, 3, 4, 5, 6
FLUID, WALL, VELOCITY, HALFWAY = 0, 1, 2, 3
Q_OF = {D2Q9: 9, D3Q19: 19}
D_OF = {D2Q9: 2, D3Q19: 3}


@dataclass
class Case:
    """A complete synthetic problem: parameters plus initial fields.

    Array layouts (x fastest): ``flags[nz][ny][nx]`` uint8,
    ``rho[C][N]``, ``u[D][N]``, optional ``df[C][Q][N]`` perturbation that is
    added to the initial equilibrium populations.
    """
    name: str
    lattice: int
    model: int
    nx: int
    ny: int
    nz: int
    tau: float
    force: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    flags: np.ndarray | None = None
    rho: np.ndarray | None = None
    u: np.ndarray | None = None
    df: np.ndarray | None = None
    mrt_rates: np.ndarray | None = None
    G: float = 0.0
    psi: int = 0
    cs_smag: float = 0.1
    u_bc: tuple = (0.0, 0.0, 0.0)
    fe: dict | None = None   # free-energy model: tau_b, tau_phi, a, kappa, gamma (tau is tau_A)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def q(self) -> int:
        return Q_OF[self.lattice]

    @property
    def d(self) -> int:
        return D_OF[self.lattice]

    @property
    def ncomp(self) -> int:
        return 2 if self.model in (SHANCHEN, FREE_ENERGY) else 1


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def rest_fields(nx, ny, nz, d, ncomp=1):
    n = nx * ny * nz
    return np.ones((ncomp, n)), np.zeros((d, n))


def channel_flags_2d(nx, ny):
    """Walls on the rows y = 0 and y = ny-1, fluid elsewhere."""
    fl = np.zeros((1, ny, nx), dtype=np.uint8)
    fl[:, 0, :] = WALL
    fl[:, ny - 1, :] = WALL
    return fl


def channel_flags_3d(nx, ny, nz):
    """Walls on the planes y = 0 and y = ny-1 (a 3-D slit channel)."""
    fl = np.zeros((nz, ny, nx), dtype=np.uint8)
    fl[:, 0, :] = WALL
    fl[:, ny - 1, :] = WALL
    return fl


def duct_flags(nx, ny, nz):
    """Walls on x = 0, x = nx-1, y = 0, y = ny-1; periodic along z."""
    fl = np.zeros((nz, ny, nx), dtype=np.uint8)
    fl[:, :, 0] = WALL
    fl[:, :, nx - 1] = WALL
    fl[:, 0, :] = WALL
    fl[:, ny - 1, :] = WALL
    return fl


def taylor_green_3d(nx, ny, nz, u0):
    """u = u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0), k = 2 pi / n per axis, rho = 1."""
    x, y, z = _grid(nx, ny, nz)
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz
    u = np.zeros((3, x.size))
    u[0] = u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    u[1] = -u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    return np.ones((1, x.size)), u


def taylor_green_2d(nx, ny, u0):
    """u = u0 (-cos kx sin ky, sin kx cos ky), rho = 1 (2-D vortex array)."""
    x, y, _ = _grid(nx, ny, 1)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    u = np.zeros((2, x.size))
    u[0] = -u0 * np.cos(kx * x) * np.sin(ky * y)
    u[1] = u0 * np.sin(kx * x) * np.cos(ky * y)
    return np.ones((1, x.size)), u


def cavity_flags(nx, ny, nz):
    """Lid-driven cavity: walls on x = nx-1, y = 0, y = ny-1, z = 0, z = nz-1; the lid
    is the rest of the plane x = 0 (velocity nodes)."""
    fl = np.zeros((nz, ny, nx), dtype=np.uint8)
    fl[:, :, 0] = VELOCITY
    fl[:, :, nx - 1] = WALL
    fl[:, 0, :] = WALL
    fl[:, ny - 1, :] = WALL
    fl[0, :, :] = WALL
    fl[nz - 1, :, :] = WALL
    return fl


def couette_flags(nx, ny, nz):
    """Plane Couette cell: velocity nodes on x = 0, walls on x = nx-1, periodic in y, z."""
    fl = np.zeros((nz, ny, nx), dtype=np.uint8)
    fl[:, :, 0] = VELOCITY
    fl[:, :, nx - 1] = WALL
    return fl


def halfway_channel_flags_2d(nx, ny):
    """Channel for half-way bounce-back: dry walls on y = 0 and y = ny-1, half-way
    bounce-back (wet) nodes on y = 1 and y = ny-2, fluid between; periodic in x."""
    fl = np.zeros((1, ny, nx), dtype=np.uint8)
    fl[:, 0, :] = WALL
    fl[:, ny - 1, :] = WALL
    fl[:, 1, :] = HALFWAY
    fl[:, ny - 2, :] = HALFWAY
    return fl


def kida_3d(n, u0):
    """Kida's vortex on a periodic n^3 grid spanning (2 pi)^3, from the paper's Kida vortex
    subsection: with (x, y, z) = 2 pi (i, j, k) / n,
    u_x = u0 sin x (cos 3y cos z - cos y cos 3z), u_y and u_z by cyclic permutation; rho = 1."""
    x, y, z = (2 * np.pi / n * a for a in _grid(n, n, n))
    u = np.empty((3, x.size))
    u[0] = u0 * np.sin(x) * (np.cos(3 * y) * np.cos(z) - np.cos(y) * np.cos(3 * z))
    u[1] = u0 * np.sin(y) * (np.cos(3 * z) * np.cos(x) - np.cos(z) * np.cos(3 * x))
    u[2] = u0 * np.sin(z) * (np.cos(3 * x) * np.cos(y) - np.cos(x) * np.cos(3 * y))
    return np.ones((1, x.size)), u


def random_state_fields(nx, ny, nz, d, seed, umax=0.05, drho=0.02, ncomp=1, stream0=0):
    """Smooth-free random macroscopic fields for parity tests (U(-umax, umax) velocity)."""
    n = nx * ny * nz
    rho = 1.0 + uniform_pm(seed, stream0 + 1, (ncomp, n), drho)
    u = uniform_pm(seed, stream0 + 2, (d, n), umax)
    return rho, u


def tau_from_nu(nu: float) -> float:
    """Relaxation time for kinematic viscosity nu in lattice units (c_s^2 = 1/3)."""
    return 0.5 + 3.0 * nu


# ---------------------------------------------------------------------------
# The five measured workloads.  ``scale`` shrinks the cubic ones for tests.

def c1_poiseuille(nx=128, ny=64, steps=2000):
    """D2Q9 BGK FP64 channel, periodic in x, walls on y=0 and y=ny-1, tau=0.8, gx=1e-6."""
    rho, u = rest_fields(nx, ny, 1, 2)
    return Case("d2q9_bgk_poiseuille_%dx%d" % (nx, ny), D2Q9, BGK, nx, ny, 1, 0.8,
                (1e-6, 0.0, 0.0), steps, channel_flags_2d(nx, ny), rho, u)


def c2_taylor_green(n=256, steps=1000, u0=0.04, nu=0.01, seed=DEFAULT_SEED, noise=1e-6):
    """D3Q19 BGK periodic Taylor-Green vortex with seeded U(+-noise) on every population."""
    rho, u = taylor_green_3d(n, n, n, u0)
    df = uniform_pm(seed, 0, (1, 19, n ** 3), noise) if noise else None
    return Case("d3q19_bgk_taylor_green_%d" % n, D3Q19, BGK, n, n, n, tau_from_nu(nu),
                (0.0, 0.0, 0.0), steps, None, rho, u, df, extra={"u0": u0, "nu": nu})


def mrt_rates_d3q19(s_nu, s_other):
    """Rates in the moment order used by the API: conserved rows 0, 3, 5, 7 get 0,
    the five stress rows 9, 11, 13, 14, 15 get s_nu, every other row s_other."""
    s = np.full(19, float(s_other))
    s[[0, 3, 5, 7]] = 0.0
    s[[9, 11, 13, 14, 15]] = float(s_nu)
    return s


def mrt_rates_d2q9(s_nu, s_other):
    s = np.full(9, float(s_other))
    s[[0, 3, 5]] = 0.0
    s[[7, 8]] = float(s_nu)
    return s


def c3_duct(nx=128, ny=128, nz=512, steps=5000, g=1e-6, s_other=1.2):
    """D3Q19 MRT square duct, walls on 4 sides, periodic along z, force g along z."""
    rho, u = rest_fields(nx, ny, nz, 3)
    return Case("d3q19_mrt_duct_%dx%dx%d" % (nx, ny, nz), D3Q19, MRT, nx, ny, nz, 0.6,
                (0.0, 0.0, g), steps, duct_flags(nx, ny, nz), rho, u,
                mrt_rates=mrt_rates_d3q19(1 / 0.6, s_other))


def c4_elbm_taylor_green(n=256, steps=1000, u0=0.05, nu=1e-5):
    """D3Q19 ELBM periodic Taylor-Green vortex at high Reynolds number."""
    rho, u = taylor_green_3d(n, n, n, u0)
    return Case("d3q19_elbm_taylor_green_%d" % n, D3Q19, ELBM, n, n, n, tau_from_nu(nu),
                (0.0, 0.0, 0.0), steps, None, rho, u, extra={"u0": u0, "nu": nu})


def kida_vortex(n=256, model=SMAG, re=1.28e5, u0=0.05, steps=1000, cs_smag=0.1):
    """D3Q19 Kida vortex, periodic n^3, Re = n u0 / nu (the paper's validation and
    lattice-performance case), run with the regularized or Smagorinsky BGK (or plain BGK)."""
    rho, u = kida_3d(n, u0)
    nu = n * u0 / re
    return Case("d3q19_kida_%d_re%g" % (n, re), D3Q19, model, n, n, n, tau_from_nu(nu), (0.0, 0.0, 0.0),
                steps, None, rho, u, cs_smag=cs_smag, extra={"u0": u0, "nu": nu, "re": re})


def lid_driven_cavity(n=254, model=BGK, re=1000.0, u_lid=0.05, steps=1000, mrt_s_other=1.2, cs_smag=0.1):
    """D3Q19 lid-driven cavity on an n^3 lattice (the paper's single-fluid benchmark
    case): full-way bounce-back walls, an equilibrium-velocity lid on x = 0 moving along
    y at u_lid, Re = u_lid (n - 2) / nu, fluid at rest."""
    rho, u = rest_fields(n, n, n, 3)
    tau = tau_from_nu(u_lid * (n - 2) / re)
    rates = mrt_rates_d3q19(1 / tau, mrt_s_other) if model == MRT else None
    return Case("d3q19_ldc_%d_re%g" % (n, re), D3Q19, model, n, n, n, tau, (0.0, 0.0, 0.0), steps,
                cavity_flags(n, n, n), rho, u, mrt_rates=rates, cs_smag=cs_smag, u_bc=(0.0, u_lid, 0.0),
                extra={"re": re, "u_lid": u_lid})


def binary_poiseuille(nx=64, ny=256, g=2e-7, nu0=1.0 / 6.0, nu1=1.0 / 24.0, kappa=1e-4, a=32e-4, gamma=25.0,
                      tau_phi=1.0, steps=0):
    """The paper's binary Poiseuille flow (free-energy model): D2Q9 channel along x with
    dry walls on y = 0, ny - 1 and half-way bounce-back nodes on y = 1, ny - 2; the core
    |y - yc| <= L/2 holds the fluid of viscosity nu1 (phi = +1, tau_A), the outer layers
    nu0 (phi = -1, tau_B); body force g along x; at rest.  yc = (ny - 1)/2 and L = yc - 1
    (the wall half a node beyond the wet node)."""
    yc = (ny - 1) / 2.0
    L = yc - 1.0
    _, y, _ = _grid(nx, ny, 1)
    phi = np.where(np.abs(y - yc) <= L / 2, 1.0, -1.0)
    rho = np.vstack([np.ones(nx * ny), phi])
    u = np.zeros((2, nx * ny))
    fe = {"tau_b": tau_from_nu(nu0), "tau_phi": tau_phi, "a": a, "kappa": kappa, "gamma": gamma}
    return Case("d2q9_binary_poiseuille_%dx%d" % (nx, ny), D2Q9, FREE_ENERGY, nx, ny, 1, tau_from_nu(nu1),
                (g, 0.0, 0.0), steps, halfway_channel_flags_2d(nx, ny), rho, u, fe=fe,
                extra={"yc": yc, "L": L, "nu0": nu0, "nu1": nu1, "g": g})


def spinodal(nx=254, ny=100, nz=100, amp=0.01, seed=DEFAULT_SEED, a=0.04, kappa=0.04, gamma=1.0, tau=1.0,
             steps=0):
    """Spinodal decomposition (the paper's binary-fluid benchmark): D3Q19 free-energy
    model, periodic, rho = 1, phi = U(-amp, amp) seeded, at rest."""
    n = nx * ny * nz
    phi = uniform_pm(seed, 3, (n,), amp)
    rho = np.vstack([np.ones(n), phi])
    fe = {"tau_b": tau, "tau_phi": tau, "a": a, "kappa": kappa, "gamma": gamma}
    return Case("d3q19_spinodal_%dx%dx%d" % (nx, ny, nz), D3Q19, FREE_ENERGY, nx, ny, nz, tau, (0.0, 0.0, 0.0),
                steps, None, rho, np.zeros((3, n)), fe=fe)


def c5_shan_chen(n=384, steps=2000, G=0.9, amp=0.01, seed=DEFAULT_SEED, tau=1.0):
    """D3Q19 two-component Shan-Chen, periodic, psi = rho, rho_A, rho_B = 1 +- amp (seeded)."""
    N = n ** 3
    rho = np.empty((2, N))
    for s in range(2):
        rho[s] = 1.0 + uniform_pm(seed, 100 + s, (N,), amp)
    u = np.zeros((3, N))
    return Case("d3q19_shan_chen_%d" % n, D3Q19, SHANCHEN, n, n, n, tau,
                (0.0, 0.0, 0.0), steps, None, rho, u, G=G, psi=0)
