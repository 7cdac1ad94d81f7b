"""Seeded synthetic inputs for the variable-density pressure solve.

This module is shared by the tests, the benchmark and the oracle checks. It
draws random numbers and evaluates closed-form synthetic fields only; it holds
none of the solver's arithmetic (no difference operator, no transform, no
tridiagonal solve, no density mixing rule). Quantities the solver derives from
these raw draws -- the right-hand side f as the discrete divergence of a face
field, and the mixture density from the colour function -- are formed by each
side with its own code.

Workloads (the paper's own validation cases are 2-D full simulations whose
fields are not published, so these stand in for them):

* ``const32``   -- 32^3 uniform grid, constant-coefficient solve; face field
  u ~ N(0,1) whose divergence is the RHS, plus one manufactured
  cos(2*pi*x) cos(4*pi*y) cos(3*pi*z/Lz) mode at cell centres.
* ``vd128``     -- 128^3 uniform, two-phase (20 spheres), 10 chained steps.
* ``mixed_tanh`` -- 256x256x512, z stretched by tanh (alpha=1.5), 200 spheres.
* ``batch``     -- 64 problems drawn from {64^3, 96x96x128, 128^3, 128x128x192}.
* ``grad256``   -- 256^3 two-phase setup plus a loss weight w ~ N(0,1).

Seeds are ``numpy.random.default_rng([200511806, config, problem, stream])``
with streams 0 = face field, 1 = spheres, 2 = temperature, 3 = p_prev,
4 = w, 5 = grid draw, 6 = finite-difference directions, 7 = target
divergence (Method III inputs: the face field is u*, the target divergence is
N(0,1) noise weighted by the gas colour with its volume-weighted mean
removed, so that a closed domain can meet it).
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_ROOT = 200511806
RHO_LIQUID = 1000.0

(STREAM_FACES, STREAM_SPHERES, STREAM_TEMP, STREAM_PPREV, STREAM_W, STREAM_GRID, STREAM_FD,
 STREAM_DIVT) = range(8)

CONFIG_IDS = {"const32": 0, "vd128": 1, "mixed_tanh": 2, "batch": 3, "grad256": 4, "method3": 5,
              "converged": 6, "bubble2d": 7}

BATCH_SHAPES = ((64, 64, 64), (96, 96, 128), (128, 128, 128), (128, 128, 192))


def rng(config: int, problem: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(config), int(problem), int(stream)])


@dataclasses.dataclass
class GridSpec:
    """Grid description handed to both sides: periodic x, y; walls in z.

    ``zf`` holds the nz+1 z-face positions (zf[0] = 0, zf[nz] = lz) or None
    for a uniform z spacing.
    """

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    zf: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def z_faces(self) -> np.ndarray:
        if self.zf is not None:
            return np.asarray(self.zf, dtype=np.float64)
        return np.arange(self.nz + 1, dtype=np.float64) * (self.lz / self.nz)

    def centres(self):
        """Cell-centre coordinates (x[nx], y[ny], z[nz])."""
        x = (np.arange(self.nx) + 0.5) * (self.lx / self.nx)
        y = (np.arange(self.ny) + 0.5) * (self.ly / self.ny)
        zf = self.z_faces()
        z = 0.5 * (zf[:-1] + zf[1:])
        return x, y, z


def tanh_faces(nz: int, lz: float, alpha: float) -> np.ndarray:
    """Wall-clustered faces: zf[k] = lz/2 * (1 + tanh(alpha (2k/nz - 1)) / tanh(alpha))."""
    s = 2.0 * np.arange(nz + 1, dtype=np.float64) / nz - 1.0
    zf = 0.5 * lz * (1.0 + np.tanh(alpha * s) / np.tanh(alpha))
    zf[0], zf[-1] = 0.0, lz
    return zf


def uniform_grid(nx: int, ny: int, nz: int) -> GridSpec:
    """Lx = Ly = 1 and Lz = nz/nx, so cells are cubes."""
    return GridSpec(nx, ny, nz, 1.0, 1.0, nz / nx, None)


def face_field(g: GridSpec, r: np.random.Generator):
    """Face-normal components u_x, u_y ~ N(0,1) on the periodic faces and u_z
    on the nz+1 z faces with u_z = 0 on both walls. Shapes: [nz,ny,nx] for x
    and y (face i+1/2 stored at i), [nz+1,ny,nx] for z (face k at zf[k])."""
    ux = r.standard_normal((g.nz, g.ny, g.nx))
    uy = r.standard_normal((g.nz, g.ny, g.nx))
    uz = r.standard_normal((g.nz + 1, g.ny, g.nx))
    uz[0] = 0.0
    uz[-1] = 0.0
    return ux, uy, uz


def manufactured_mode(g: GridSpec, a: int = 1, b: int = 2, m: int = 3) -> np.ndarray:
    """cos(2 pi a x/Lx) cos(2 pi b y/Ly) cos(pi m z/Lz) at cell centres."""
    x, y, z = g.centres()
    cx = np.cos(2.0 * np.pi * a * x / g.lx)
    cy = np.cos(2.0 * np.pi * b * y / g.ly)
    cz = np.cos(np.pi * m * z / g.lz)
    return cz[:, None, None] * cy[None, :, None] * cx[None, None, :]


def _separable_sum(g: GridSpec, amp, kx, ky, kz, phx, phy) -> np.ndarray:
    """sum_t amp_t cos(2 pi kx_t x/Lx + phx_t) cos(2 pi ky_t y/Ly + phy_t) cos(pi kz_t z/Lz)."""
    x, y, z = g.centres()
    cx = np.cos(2.0 * np.pi * np.outer(kx, x) / g.lx + phx[:, None])  # [T, nx]
    cy = np.cos(2.0 * np.pi * np.outer(ky, y) / g.ly + phy[:, None])  # [T, ny]
    cz = np.cos(np.pi * np.outer(kz, z) / g.lz) * amp[:, None]        # [T, nz]
    xy = (cy[:, :, None] * cx[:, None, :]).reshape(len(amp), g.ny * g.nx)
    return (cz.T @ xy).reshape(g.nz, g.ny, g.nx)


def temperature_field(g: GridSpec, r: np.random.Generator) -> np.ndarray:
    """Smooth field theta in [0, 1]: 64 random cosine modes (a, b, m in 0..3)."""
    a, b, m = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    a, b, m = a.ravel(), b.ravel(), m.ravel()
    amp = r.standard_normal(a.size)
    phx = r.uniform(0.0, 2.0 * np.pi, a.size)
    phy = r.uniform(0.0, 2.0 * np.pi, a.size)
    th = _separable_sum(g, amp, a, b, m, phx, phy)
    lo, hi = th.min(), th.max()
    return (th - lo) / (hi - lo)


def previous_pressure(g: GridSpec, r: np.random.Generator) -> np.ndarray:
    """Smooth p_prev with zero wall-normal derivative: 125 modes (0..4)^3,
    amplitude N(0,1)/(1 + a^2 + b^2 + m^2)."""
    a, b, m = np.meshgrid(np.arange(5), np.arange(5), np.arange(5), indexing="ij")
    a, b, m = a.ravel(), b.ravel(), m.ravel()
    amp = r.standard_normal(a.size) / (1.0 + a * a + b * b + m * m)
    phx = r.uniform(0.0, 2.0 * np.pi, a.size)
    phy = r.uniform(0.0, 2.0 * np.pi, a.size)
    return _separable_sum(g, amp, a, b, m, phx, phy)


def colour_spheres(g: GridSpec, r: np.random.Generator, n_spheres: int) -> np.ndarray:
    """Colour function Phi (1 = gas) of n smoothed spheres.

    Radius R ~ U(0.05, 0.15) Lx; centre x, y ~ U(0, L), z ~ U(R, Lz - R);
    signed distance d with the minimum image in x and y;
    Phi = max over spheres of (1 - tanh(d/eps))/2, eps = 1.5 dx. Cells farther
    than 12 eps outside a sphere take no contribution from it (the profile is
    below 4e-11 there)."""
    x, y, z = g.centres()
    dx = g.lx / g.nx
    eps = 1.5 * dx
    cut = 12.0 * eps
    phi = np.zeros((g.nz, g.ny, g.nx))
    rad = r.uniform(0.05, 0.15, n_spheres) * g.lx
    cxs = r.uniform(0.0, g.lx, n_spheres)
    cys = r.uniform(0.0, g.ly, n_spheres)
    czs = r.uniform(0.0, 1.0, n_spheres)
    zf = g.z_faces()
    for s in range(n_spheres):
        R = rad[s]
        cz = R + czs[s] * (g.lz - 2.0 * R)
        reach = R + cut
        # x and y index windows (periodic), z window (clipped)
        ix = np.arange(int(np.floor((cxs[s] - reach) / dx)) - 1, int(np.ceil((cxs[s] + reach) / dx)) + 2)
        iy = np.arange(int(np.floor((cys[s] - reach) / (g.ly / g.ny))) - 1,
                       int(np.ceil((cys[s] + reach) / (g.ly / g.ny))) + 2)
        ix = np.unique(np.mod(ix, g.nx))
        iy = np.unique(np.mod(iy, g.ny))
        k0 = max(int(np.searchsorted(zf, cz - reach)) - 1, 0)
        k1 = min(int(np.searchsorted(zf, cz + reach)) + 1, g.nz)
        iz = np.arange(k0, k1)
        ddx = x[ix] - cxs[s]
        ddx -= g.lx * np.round(ddx / g.lx)
        ddy = y[iy] - cys[s]
        ddy -= g.ly * np.round(ddy / g.ly)
        ddz = z[iz] - cz
        d = np.sqrt(ddz[:, None, None] ** 2 + ddy[None, :, None] ** 2 + ddx[None, None, :] ** 2) - R
        val = np.where(d < cut, 0.5 * (1.0 - np.tanh(d / eps)), 0.0)
        sub = phi[np.ix_(iz, iy, ix)]
        phi[np.ix_(iz, iy, ix)] = np.maximum(sub, val)
    return phi


@dataclasses.dataclass
class Case:
    """Raw inputs of one problem. ``phi`` and ``rho_gas`` give the mixture
    density rho = rho_gas*Phi + rho_liq*(1-Phi); ``faces`` give the RHS as the
    discrete divergence; ``extra_rhs`` (if not None) is added to that RHS."""

    name: str
    grid: GridSpec
    faces: tuple
    extra_rhs: np.ndarray | None
    phi: np.ndarray | None
    rho_gas: np.ndarray | None
    rho_liq: float
    p_prev: np.ndarray | None
    w: np.ndarray | None
    n_steps: int


def _two_phase(g: GridSpec, config: int, problem: int, n_spheres: int):
    phi = colour_spheres(g, rng(config, problem, STREAM_SPHERES), n_spheres)
    theta = temperature_field(g, rng(config, problem, STREAM_TEMP))
    rho_gas = 1.0 + 4.0 * theta
    p_prev = previous_pressure(g, rng(config, problem, STREAM_PPREV))
    return phi, rho_gas, p_prev


def two_phase_case(name: str, g: GridSpec, config: int, problem: int = 0, n_spheres: int = 20,
                   n_steps: int = 1, with_w: bool = False) -> Case:
    faces = face_field(g, rng(config, problem, STREAM_FACES))
    phi, rho_gas, p_prev = _two_phase(g, config, problem, n_spheres)
    w = rng(config, problem, STREAM_W).standard_normal((g.nz, g.ny, g.nx)) if with_w else None
    return Case(name, g, faces, None, phi, rho_gas, RHO_LIQUID, p_prev, w, n_steps)


def const32(n: int = 32) -> Case:
    g = uniform_grid(n, n, n)
    faces = face_field(g, rng(0, 0, STREAM_FACES))
    return Case("const32", g, faces, manufactured_mode(g), None, None, RHO_LIQUID, None, None, 1)


def vd128(n: int = 128, n_steps: int = 10) -> Case:
    return two_phase_case("vd128", uniform_grid(n, n, n), 1, 0, 20, n_steps)


def mixed_tanh(nx: int = 256, ny: int = 256, nz: int = 512, n_spheres: int = 200) -> Case:
    g = GridSpec(nx, ny, nz, 1.0, 1.0, 2.0, tanh_faces(nz, 2.0, 1.5))
    return two_phase_case("mixed_tanh", g, 2, 0, n_spheres, 1)


def grad256(n: int = 256) -> Case:
    return two_phase_case("grad256", uniform_grid(n, n, n), 4, 0, 20, 1, with_w=True)


def batch_shapes(n_problems: int = 64, shapes=BATCH_SHAPES) -> list:
    """Per-problem grid shapes drawn uniformly from ``shapes``."""
    r = rng(3, 0, STREAM_GRID)
    idx = r.integers(0, len(shapes), n_problems)
    return [shapes[i] for i in idx]


def batch(n_problems: int = 64, shapes=BATCH_SHAPES) -> list:
    out = []
    for p, (nx, ny, nz) in enumerate(batch_shapes(n_problems, shapes)):
        out.append(two_phase_case(f"batch{p}", uniform_grid(nx, ny, nz), 3, p, 20, 1))
    return out


@dataclasses.dataclass
class Method3Case:
    """Inputs of a Method-III solve: ``base.faces`` is the predicted velocity
    u*, ``div_target`` the target divergence, ``dt`` the time step; the
    density comes from ``base`` as for Method I."""

    base: Case
    div_target: np.ndarray
    dt: float


def target_divergence(g: GridSpec, phi: np.ndarray, r: np.random.Generator,
                      scale: float = 1.0) -> np.ndarray:
    """scale * Phi * N(0,1), minus its volume-weighted mean."""
    d = scale * phi * r.standard_normal((g.nz, g.ny, g.nx))
    h = np.diff(g.z_faces())
    v = np.broadcast_to(h[:, None, None], d.shape)
    return d - (v * d).sum() / v.sum()


def method3_case(name: str, g: GridSpec, problem: int = 0, n_spheres: int = 20,
                 dt: float = 1e-3, rho_liq: float = 10.0) -> Method3Case:
    """Two-phase Method-III inputs; the liquid density defaults to 10 (density
    ratio up to 10 against gas at 1-5), the rising-bubble ratio."""
    base = dataclasses.replace(two_phase_case(name, g, CONFIG_IDS["method3"], problem, n_spheres),
                               rho_liq=rho_liq)
    dtg = target_divergence(g, base.phi, rng(CONFIG_IDS["method3"], problem, STREAM_DIVT))
    return Method3Case(base, dtg, dt)


def method3_128(n: int = 128) -> Method3Case:
    return method3_case("method3_128", uniform_grid(n, n, n), 0, 20)


def converged_case(name: str, g: GridSpec, problem: int = 0, n_spheres: int = 20,
                   rho_liq: float = 10.0) -> Case:
    """Two-phase inputs of the converged variable-density solve and its
    adjoint (right-hand side from the face field, seed w for the loss
    sum(w p)), liquid density 10 as for Method III."""
    return dataclasses.replace(
        two_phase_case(name, g, CONFIG_IDS["converged"], problem, n_spheres, 1, with_w=True),
        rho_liq=rho_liq)


def converged_128(n: int = 128) -> Case:
    return converged_case("converged_128", uniform_grid(n, n, n), 0, 20)


def rising_bubble_2d(nx: int = 128, nz: int = 256, rho_liq: float = 10.0,
                     problem: int = 0) -> Case:
    """Frozen snapshot shaped like the paper's rising-bubble case C2 (Sec. 4):
    an x-z domain 1 x 2 (x periodic, walls in z, ny = 1), one circular gas
    bubble of diameter 0.5 centred at (0.5, 0.5), Phi = (1 - tanh(d/eps))/2
    with d the signed distance to the circle and eps = 1.5 dx, gas density 1
    and liquid density rho_liq (density ratio 10 for the paper's first
    temperature ratio). The right-hand side is the divergence of the seeded
    face field; nothing of the paper's flow state is reproduced."""
    g = GridSpec(nx, 1, nz, 1.0, 1.0 / nx, 2.0, None)
    x, _, z = g.centres()
    eps = 1.5 * g.lx / nx
    d = np.sqrt((z[:, None, None] - 0.5) ** 2 + (x[None, None, :] - 0.5) ** 2) - 0.25
    phi = 0.5 * (1.0 - np.tanh(d / eps))
    faces = face_field(g, rng(CONFIG_IDS["bubble2d"], problem, STREAM_FACES))
    return Case("rising_bubble_2d", g, faces, None, phi, np.ones((nz, 1, nx)), rho_liq, None,
                None, 1)


def fd_directions(config: int, n_dirs: int, shape) -> np.ndarray:
    return rng(config, 0, STREAM_FD).standard_normal((n_dirs,) + tuple(shape))
