"""Seeded synthetic initial conditions for the 3D Newtonian adiabatic hydro update.

This module only builds input states. It holds none of the solver's arithmetic
(no cons-to-prim, reconstruction, Riemann solve, update or time-step rule), so
both the GPU path and the CPU reference solver under ``oracle/`` can take their
inputs from it without sharing any of the method.

Every generator returns a :class:`Problem`: the conserved state
``U[5][nz][ny][nx]`` (float64, x fastest, variables rho, Mx, My, Mz, E) plus
the mesh, boundary and gas parameters that define the run. Conserved variables
follow the paper's definition of the Newtonian hydro state (Sec. 3.1, Eq. 4):
U = [rho, rho v, E] with E = u_g + rho v^2 / 2 and the gamma-law EOS
p = (gamma - 1) u_g.

Random draws are either made once for the whole grid with a seeded numpy
generator (turbulence modes, Sedov centre, Sod axis) or by a counter-based hash
of (seed, global cell index) (KH noise), so that a state is identical whether it
is generated whole or cut into MeshBlocks afterwards.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

PERIODIC = 0
OUTFLOW = 1
PLM = 0
PPM4 = 1
WENOZ = 2
PPMX = 3
FP64 = 0
MIXED = 1

# Ghost depth each reconstruction needs: PLM reads c-1..c+1 of a cell, so a face
# needs two cells on each side; PPM4 (Colella & Woodward 1984), PPMX and WENO-Z
# (c-2..c+2 of a cell) need three.
NGHOST = {PLM: 2, PPM4: 3, WENOZ: 3, PPMX: 3}


@dataclass
class Problem:
    """A hydro problem: mesh, boundaries, gas and algorithm choices, and U."""

    n: tuple                      # (nx, ny, nz) interior cells of the global mesh
    lo: tuple                     # (x0, y0, z0) lower domain corner
    hi: tuple                     # (x1, y1, z1) upper domain corner
    bc: tuple                     # ((xl, xu), (yl, yu), (zl, zu)), PERIODIC/OUTFLOW
    U: np.ndarray                 # float64 [5][nz][ny][nx]
    gamma: float = 5.0 / 3.0
    cfl: float = 0.3
    recon: int = PLM
    precision: int = FP64
    block: tuple | None = None    # MeshBlock interior size (bx, by, bz)
    rho_floor: float = 1e-10
    p_floor: float = 1e-13
    fofc: int = 0                 # first-order flux correction (Sec. 3) on/off
    rk: int = 2                   # SSP-RK order (Sec. 3): 1, 2, 3 or 4 (SSPRK(10,4))
    refine: tuple | None = None   # ((lo), (hi)) root blocks refined once, or a tuple of
                                  # such boxes (their union is refined); U is then
                                  # leaf-major [leaf][5][bz][by][bx] (see to_leaves)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dx(self):
        """Cell widths of the root (level-0) grid."""
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))

    @property
    def cells(self):
        if self.refine is not None:
            return int(self.U.shape[0]) * int(np.prod(self.block))
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def with_(self, **kw):
        return replace(self, **kw)


# --------------------------------------------------------------------------
# Counter-based random numbers
# --------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter) -> np.ndarray:
    """Output number ``counter + 1`` of a SplitMix64 generator seeded with ``seed``.

    SplitMix64 (Steele, Lea & Flood 2014; the variant published by Vigna) adds
    the golden-ratio increment to its state once per draw and scrambles the
    state with two xor-shift-multiply rounds. Evaluating it at an arbitrary
    counter makes it a stateless hash of (seed, counter). Returns uint64.
    """
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counter) -> np.ndarray:
    """SplitMix64 output mapped to [0, 1) as r / 2^64 (top 53 bits, exact)."""
    z = splitmix64(seed, counter)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# Helpers
# --------------------------------------------------------------------------
def _centres(n, lo, hi):
    d = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * d


def conserved(rho, vx, vy, vz, p, gamma):
    """Build U = [rho, rho v, p/(gamma-1) + rho v^2 / 2] (Sec. 3.1, Eq. 4)."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast(rho, vx, vy, vz, p).shape
    U = np.empty((5,) + shape, dtype=np.float64)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return U


def _default_block(n, want=64):
    """Largest MeshBlock edge <= ``want`` that divides each mesh dimension."""
    out = []
    for nd in n:
        b = min(nd, want)
        while nd % b:
            b -= 1
        out.append(b)
    return tuple(out)


# --------------------------------------------------------------------------
# Uniform state
# --------------------------------------------------------------------------
def uniform(n=(16, 16, 16), rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, gamma=5.0 / 3.0,
            bc=PERIODIC, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), **kw):
    nx, ny, nz = n
    shape = (nz, ny, nx)
    U = conserved(np.full(shape, rho), np.full(shape, v[0]), np.full(shape, v[1]),
                  np.full(shape, v[2]), np.full(shape, p), gamma)
    bcs = tuple((bc, bc) for _ in range(3))
    return Problem(n=tuple(n), lo=tuple(lo), hi=tuple(hi), bc=bcs, U=U,
                   gamma=gamma, name="uniform", **kw)


# --------------------------------------------------------------------------
# Linear sound-wave eigenmode along the grid diagonal
# --------------------------------------------------------------------------
def sound_wave(N=32, amp=1e-6, t=0.0, n=None, rho0=1.0, p0=0.6, gamma=5.0 / 3.0,
               wavevec=(1, 1, 1), **kw):
    """Cell-averaged right-going sound eigenmode on the periodic unit cube.

    The paper's convergence and performance tests propagate an exact linear
    eigenmode for one wave period (Sec. 3.1, linear-wave test; Sec. 5.1,
    Table 1 workload). With background (rho0, p0, v = 0), sound speed
    c = sqrt(gamma p0 / rho0), total enthalpy H = (E0 + p0)/rho0 and
    wave vector k = 2 pi ``wavevec``, the conserved state is
        U(x, t) = U0 + amp * [1, c k^, H] * sin(k.x - c |k| t).
    Each cell holds the exact average over the cell, which for a product of
    per-axis phases is the centre value times prod_d sinc(k_d dx_d / 2).
    ``t`` > 0 gives the exact linear solution at that time.
    """
    if n is None:
        n = (N, N, N)
    nx, ny, nz = n
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    kv = 2.0 * np.pi * np.asarray(wavevec, dtype=np.float64)
    kmag = float(np.sqrt(kv @ kv))
    khat = kv / kmag
    c = np.sqrt(gamma * p0 / rho0)
    E0 = p0 / (gamma - 1.0)
    H = (E0 + p0) / rho0
    omega = c * kmag
    dx = [(hi[d] - lo[d]) / n[d] for d in range(3)]
    x = _centres(nx, lo[0], hi[0])
    y = _centres(ny, lo[1], hi[1])
    z = _centres(nz, lo[2], hi[2])
    phase = (kv[0] * x[None, None, :] + kv[1] * y[None, :, None]
             + kv[2] * z[:, None, None] - omega * t)
    damp = 1.0
    for d in range(3):
        a = 0.5 * kv[d] * dx[d]
        damp *= np.sin(a) / a if a != 0.0 else 1.0
    s = np.sin(phase) * damp
    U = np.empty((5, nz, ny, nx), dtype=np.float64)
    U[0] = rho0 + amp * s
    U[1] = amp * c * khat[0] * s
    U[2] = amp * c * khat[1] * s
    U[3] = amp * c * khat[2] * s
    U[4] = E0 + amp * H * s
    bcs = ((PERIODIC, PERIODIC),) * 3
    period = 2.0 * np.pi / omega
    return Problem(n=tuple(n), lo=lo, hi=hi, bc=bcs, U=U, gamma=gamma,
                   name="sound_wave",
                   meta=dict(amp=amp, period=period, rho0=rho0, p0=p0, t=t,
                             wavevec=tuple(wavevec)), **kw)


# --------------------------------------------------------------------------
# Solenoidal turbulent velocity field
# --------------------------------------------------------------------------
def turbulence(N=256, seed=1, kmin=1, kmax=16, mach=0.5, rho=1.0, p=1.0,
               gamma=5.0 / 3.0, **kw):
    """Random-phase solenoidal velocity field with a k^-5/3 shell spectrum.

    Every integer wave vector with kmin <= |k| <= kmax gets amplitude
    |k|^(-11/6) (so the energy per shell scales as k^-5/3), a uniform random
    phase and a random unit direction perpendicular to k. The field is the
    real part of the Hermitian-symmetric inverse FFT on an N^3 grid, rescaled
    so that the rms speed is ``mach`` times the sound speed. Density and
    pressure are uniform. The draws come from numpy's PCG64 seeded with
    ``seed`` in a fixed mode order, and the field is built whole, so any
    MeshBlock decomposition sees the same state.
    """
    rng = np.random.default_rng(seed)
    K = np.arange(-kmax, kmax + 1)
    kx, ky, kz = np.meshgrid(K, K, K, indexing="ij")
    kk = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    k2 = (kk * kk).sum(1)
    sel = (k2 >= kmin * kmin) & (k2 <= kmax * kmax)
    kk = kk[sel]
    # keep one of each +-k pair: first nonzero component positive
    first = np.where(kk[:, 0] != 0, kk[:, 0], np.where(kk[:, 1] != 0, kk[:, 1], kk[:, 2]))
    kk = kk[first > 0]
    nm = kk.shape[0]
    kmag = np.sqrt((kk * kk).sum(1).astype(np.float64))
    amp = kmag ** (-11.0 / 6.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=nm)
    # random unit direction perpendicular to k: isotropic draw, project, normalise
    g = rng.normal(size=(nm, 3))
    khat = kk / kmag[:, None]
    g -= (g * khat).sum(1)[:, None] * khat
    g /= np.sqrt((g * g).sum(1))[:, None]
    spec = np.zeros((3, N, N, N), dtype=np.complex128)
    coef = (amp * np.exp(1j * phase))[:, None] * g        # (nm, 3)
    ix = np.mod(kk[:, 0], N)
    iy = np.mod(kk[:, 1], N)
    iz = np.mod(kk[:, 2], N)
    jx = np.mod(-kk[:, 0], N)
    jy = np.mod(-kk[:, 1], N)
    jz = np.mod(-kk[:, 2], N)
    for c in range(3):
        # array axes are (z, y, x); wave vector components are (x, y, z)
        spec[c, iz, iy, ix] = 0.5 * coef[:, c]
        spec[c, jz, jy, jx] = 0.5 * np.conj(coef[:, c])
    v = np.fft.ifftn(spec, axes=(1, 2, 3)).real * (N ** 3)
    del spec
    cs = np.sqrt(gamma * p / rho)
    rms = np.sqrt(np.mean((v * v).sum(0)))
    v *= (mach * cs) / rms
    U = conserved(np.full((N, N, N), rho), v[0], v[1], v[2], np.full((N, N, N), p), gamma)
    bcs = ((PERIODIC, PERIODIC),) * 3
    return Problem(n=(N, N, N), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bcs, U=U,
                   gamma=gamma, name="turbulence",
                   meta=dict(seed=seed, kmin=kmin, kmax=kmax, mach=mach), **kw)


# --------------------------------------------------------------------------
# Kelvin-Helmholtz shear layer
# --------------------------------------------------------------------------
def kelvin_helmholtz(N=512, seed=2, n=None, gamma=5.0 / 3.0, noise=1e-2, bg_noise=0.0, **kw):
    """Sharp double shear layer on [-1/2, 1/2]^3 with seeded vy noise.

    |y| < 1/4: rho = 2, vx = +1/2; elsewhere rho = 1, vx = -1/2; p = 2.5.
    Where ||y| - 1/4| < 0.05, vy = noise * (2 r - 1) with r the SplitMix64
    draw for (seed, global cell index i + nx (j + ny k)). ``bg_noise`` > 0
    also multiplies rho, vx and p everywhere by independent factors
    1 + bg_noise (2 r - 1) (counters offset by 1, 2 and 3 times the cell
    count), so that no two cells hold exactly equal values.
    """
    if n is None:
        n = (N, N, N)
    nx, ny, nz = n
    lo, hi = (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5)
    y = _centres(ny, lo[1], hi[1])
    inner = np.abs(y) < 0.25
    rho_y = np.where(inner, 2.0, 1.0)
    vx_y = np.where(inner, 0.5, -0.5)
    band = np.abs(np.abs(y) - 0.25) < 0.05
    shape = (nz, ny, nx)
    rho = np.broadcast_to(rho_y[None, :, None], shape)
    vx = np.broadcast_to(vx_y[None, :, None], shape)
    vy = np.zeros(shape)
    rows = np.nonzero(band)[0]
    if rows.size:  # hash only the band rows; the cell index is the global one
        k = np.arange(nz, dtype=np.uint64)[:, None, None]
        j = rows.astype(np.uint64)[None, :, None]
        i = np.arange(nx, dtype=np.uint64)[None, None, :]
        idx = i + np.uint64(nx) * (j + np.uint64(ny) * k)
        vy[:, rows, :] = noise * (2.0 * uniform01(seed, idx) - 1.0)
    pres = np.full(shape, 2.5)
    if bg_noise > 0.0:
        ncell = nx * ny * nz
        idx = np.arange(ncell, dtype=np.uint64).reshape(shape)
        fac = [1.0 + bg_noise * (2.0 * uniform01(seed, idx + np.uint64(m * ncell)) - 1.0)
               for m in (1, 2, 3)]
        rho, vx, pres = rho * fac[0], vx * fac[1], pres * fac[2]
    U = conserved(rho, vx, vy, 0.0, pres, gamma)
    bcs = ((PERIODIC, PERIODIC),) * 3
    return Problem(n=tuple(n), lo=lo, hi=hi, bc=bcs, U=U, gamma=gamma,
                   name="kelvin_helmholtz", meta=dict(seed=seed), **kw)


# --------------------------------------------------------------------------
# Sedov blast
# --------------------------------------------------------------------------
def sedov(N=32, seed=3, energy=1.0, radius_cells=3.0, rho=1.0, p=1e-5,
          gamma=5.0 / 3.0, centre=None, noise=0.0, **kw):
    """Point explosion on the unit cube with outflow boundaries.

    Background rho = 1, p = 1e-5, v = 0. The centre is a seeded cell centre at
    least four cells from every face; ``energy`` is spread evenly, as internal
    energy, over the cells whose centres lie within ``radius_cells`` cell
    widths of it (123 cells for radius 3), replacing the background there.
    ``noise`` > 0 multiplies the density and the pressure by independent
    factors 1 + noise (2 r - 1), r from SplitMix64(seed, counter) with counter
    = global cell index (density) and N^3 + global cell index (pressure),
    which breaks the exact mirror symmetry of the blast.
    """
    if centre is None:
        rng = np.random.default_rng(seed)
        centre = tuple(int(c) for c in rng.integers(4, N - 4, size=3))
    cx, cy, cz = centre
    dx = 1.0 / N
    shape = (N, N, N)
    i = np.arange(N)
    di = (i - cx)[None, None, :]
    dj = (i - cy)[None, :, None]
    dk = (i - cz)[:, None, None]
    inside = (di * di + dj * dj + dk * dk) <= radius_cells * radius_cells
    ncell = int(inside.sum())
    u_in = energy / (ncell * dx ** 3)
    pres = np.where(inside, (gamma - 1.0) * u_in, p)
    dens = np.full(shape, rho)
    if noise > 0.0:
        idx = np.arange(N * N * N, dtype=np.uint64).reshape(shape)
        dens = dens * (1.0 + noise * (2.0 * uniform01(seed, idx) - 1.0))
        pres = pres * (1.0 + noise * (2.0 * uniform01(seed, idx + np.uint64(N * N * N)) - 1.0))
    U = conserved(dens, 0.0, 0.0, 0.0, pres, gamma)
    bcs = ((OUTFLOW, OUTFLOW),) * 3
    return Problem(n=(N, N, N), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bcs, U=U,
                   gamma=gamma, name="sedov",
                   meta=dict(seed=seed, centre=(cx, cy, cz), ncell=ncell,
                             energy=energy, rho=rho), **kw)


# --------------------------------------------------------------------------
# Sod shock tube
# --------------------------------------------------------------------------
def sod(N=128, axis=None, seed=4, ntrans=None, gamma=5.0 / 3.0, x0=0.5, **kw):
    """Sod's shock tube along ``axis`` (seeded if None) on [0, 1], outflow.

    Left (coordinate < x0): rho = 1, p = 1; right: rho = 0.125, p = 0.1; v = 0.
    Transverse axes hold ``ntrans`` cells (default N) of the same state.
    """
    if axis is None:
        axis = int(np.random.default_rng(seed).integers(0, 3))
    if ntrans is None:
        ntrans = N
    n = [ntrans, ntrans, ntrans]
    n[axis] = N
    nx, ny, nz = n
    xc = _centres(N, 0.0, 1.0)
    left = xc < x0
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    shape = (nz, ny, nx)
    view = [1, 1, 1]
    view[2 - axis] = N
    rho = np.broadcast_to(rho1.reshape(view), shape)
    p = np.broadcast_to(p1.reshape(view), shape)
    U = conserved(rho, 0.0, 0.0, 0.0, p, gamma)
    bcs = ((OUTFLOW, OUTFLOW),) * 3
    return Problem(n=tuple(n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bcs, U=U,
                   gamma=gamma, name="sod", meta=dict(axis=axis, x0=x0), **kw)


def entropy_wave(N=32, amp=0.2, v0=1.0, p0=1.0, rho0=1.0, t=0.0, axis=0, ntrans=1,
                 gamma=5.0 / 3.0, **kw):
    """Cell-averaged entropy (density) wave advected at ``v0`` along ``axis``
    of the periodic unit domain, with uniform pressure and velocity.

    The paper's linear-wave tests cover entropy waves beside sound waves
    (Sec. 3.1). With uniform p and v the Euler equations reduce exactly to
    advection of rho, so rho(x, t) = rho0 + amp sin(2 pi (x - v0 t)) for any
    amplitude. Momentum and energy are linear in rho at fixed (v, p), so each
    cell holds the exact average: the centre value times sinc(pi dx).
    ``t`` > 0 gives the exact solution at that time.
    """
    n = [ntrans, ntrans, ntrans]
    n[axis] = N
    nx, ny, nz = n
    xc = _centres(N, 0.0, 1.0)
    h = 1.0 / N
    a = np.pi * h
    rho1 = rho0 + amp * np.sin(2.0 * np.pi * (xc - v0 * t)) * (np.sin(a) / a)
    view = [1, 1, 1]
    view[2 - axis] = N
    rho = np.broadcast_to(rho1.reshape(view), (nz, ny, nx))
    v = [0.0, 0.0, 0.0]
    v[axis] = v0
    U = np.empty((5, nz, ny, nx), dtype=np.float64)
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * v[d]
    U[4] = p0 / (gamma - 1.0) + 0.5 * rho * (v0 * v0)
    bcs = ((PERIODIC, PERIODIC),) * 3
    return Problem(n=tuple(n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=bcs, U=U,
                   gamma=gamma, name="entropy_wave",
                   meta=dict(period=1.0 / abs(v0), axis=axis, amp=amp), **kw)


def shu_osher(N=200, axis=0, ntrans=1, gamma=1.4, **kw):
    """Shu & Osher's shock-entropy interaction (the paper's Fig. 2 right panel
    shows it): on [-5, 5], a Mach-3 shock at x = -4 moves right into
    rho = 1 + 0.2 sin(5x), p = 1, v = 0; the post-shock state is
    (rho, v, p) = (3.857143, 2.629369, 10.33333). Cell-centre point values,
    outflow boundaries, gamma = 1.4; the customary end time is 1.8.
    """
    n = [ntrans, ntrans, ntrans]
    n[axis] = N
    nx, ny, nz = n
    xc = _centres(N, -5.0, 5.0)
    post = xc < -4.0
    rho1 = np.where(post, 3.857143, 1.0 + 0.2 * np.sin(5.0 * xc))
    v1 = np.where(post, 2.629369, 0.0)
    p1 = np.where(post, 10.33333, 1.0)
    view = [1, 1, 1]
    view[2 - axis] = N
    shape = (nz, ny, nx)
    rho = np.broadcast_to(rho1.reshape(view), shape)
    vel = np.broadcast_to(v1.reshape(view), shape)
    p = np.broadcast_to(p1.reshape(view), shape)
    v = [0.0, 0.0, 0.0]
    v[axis] = vel
    U = conserved(rho, v[0], v[1], v[2], p, gamma)
    lo, hi = [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]
    lo[axis], hi[axis] = -5.0, 5.0
    for d in range(3):
        if d != axis:
            hi[d] = 10.0 / N
    bcs = ((OUTFLOW, OUTFLOW),) * 3
    return Problem(n=tuple(n), lo=tuple(lo), hi=tuple(hi), bc=bcs, U=U, gamma=gamma,
                   name="shu_osher", meta=dict(axis=axis, t_end=1.8), **kw)


# --------------------------------------------------------------------------
# The five workloads (sizes, steps and choices as the benchmark defines them)
# --------------------------------------------------------------------------
def workload_eigenmode_32():
    """32^3 single MeshBlock, amplitude 1e-6 diagonal sound wave, PLM, FP64, 10 steps."""
    pb = sound_wave(N=32, amp=1e-6)
    return pb.with_(block=(32, 32, 32), recon=PLM, precision=FP64), 10


def workload_turbulence_256(precision=FP64, N=256, block=64):
    """256^3 periodic turbulence in 64 MeshBlocks of 64^3, PLM, 20 steps."""
    pb = turbulence(N=N, seed=1)
    return pb.with_(block=(block,) * 3, recon=PLM, precision=precision), 20


def workload_kh_512(precision=FP64, N=512, block=128):
    """512^3 periodic KH layer in 64 MeshBlocks of 128^3, PPM4, 10 steps."""
    pb = kelvin_helmholtz(N=N, seed=2)
    return pb.with_(block=(block,) * 3, recon=PPM4, precision=precision), 10


def inject_to_leaves(pb, box, leaves):
    """Refined version of a uniform problem: coarse leaves keep their blocks;
    each fine leaf repeats its parent's cells 2 x 2 x 2 (a piecewise-constant
    fine state with the same cell averages), built leaf by leaf."""
    bx, by, bz = (int(b) for b in pb.block)
    lv = np.asarray(leaves).reshape(-1, 4)
    out = np.empty((len(lv), 5, bz, by, bx), dtype=np.float64)
    for q, (L, lx, ly, lz) in enumerate(lv):
        if L == 0:
            out[q] = pb.U[:, lz * bz:(lz + 1) * bz, ly * by:(ly + 1) * by, lx * bx:(lx + 1) * bx]
            continue
        x0, y0, z0 = lx * bx // 2, ly * by // 2, lz * bz // 2
        par = pb.U[:, z0:z0 + bz // 2, y0:y0 + by // 2, x0:x0 + bx // 2]
        out[q] = par.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    return pb.with_(U=out, refine=(tuple(box[0]), tuple(box[1])),
                    name=(pb.name + " refined").strip())


REFINED_BOX_256 = ((1, 1, 1), (3, 3, 3))


def workload_turbulence_refined(leaves, precision=FP64, N=256, block=64, box=REFINED_BOX_256):
    """The 256^3 turbulence workload with its central 2 x 2 x 2 root blocks
    refined once: 56 MeshBlocks of 64^3 on level 0 and 64 on level 1 (31.5 M
    cells), PLM, 20 steps; fine leaves start from their parents' cells.
    ``leaves`` is the solver's leaf order for this mesh."""
    pb, steps = workload_turbulence_256(precision=precision, N=N, block=block)
    return inject_to_leaves(pb, box, leaves), steps


SEDOV_SIZES = (32, 48, 64, 96, 128)


def workload_sedov_batch(count=48, seed=3, sizes=SEDOV_SIZES, precision=MIXED):
    """``count`` Sedov problems with seeded sizes, outflow, PLM, 50 steps each."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sizes), size=count)
    out = []
    for q, N in enumerate(Ns):
        N = int(N)
        pb = sedov(N=N, seed=seed * 1000 + q)
        out.append(pb.with_(block=_default_block((N, N, N)), recon=PLM, precision=precision))
    return out, 50


SERVE_TYPES = ("sod", "kh", "sedov")
SERVE_SIZES = (32, 48, 64, 96, 128, 192, 256)
SERVE_STEPS = (10, 20, 50, 100, 200)


def serving_request(seed: int, index: int, max_n: int | None = None, generate: bool = True):
    """Request ``index`` of the seeded serving stream: (problem, steps).

    Type, size, step count and precision are each uniform over their grids
    (``max_n`` drops larger sizes from the size grid); the draws for one
    request depend only on (seed, index). With ``generate=False`` the problem
    carries no state yet (``U is None``): ``generate_state`` builds it.
    """
    r = uniform01(seed, np.arange(4, dtype=np.uint64) + np.uint64(4 * index))
    typ = SERVE_TYPES[int(r[0] * len(SERVE_TYPES))]
    sizes = SERVE_SIZES if max_n is None else tuple(x for x in SERVE_SIZES if x <= max_n)
    N = sizes[int(r[1] * len(sizes))]
    steps = SERVE_STEPS[int(r[2] * len(SERVE_STEPS))]
    prec = FP64 if r[3] < 0.5 else MIXED
    sub = seed * 1_000_003 + index
    if typ == "kh":
        lo, hi, bc = (-0.5,) * 3, (0.5,) * 3, ((PERIODIC, PERIODIC),) * 3
    else:
        lo, hi, bc = (0.0,) * 3, (1.0,) * 3, ((OUTFLOW, OUTFLOW),) * 3
    pb = Problem(n=(N, N, N), lo=lo, hi=hi, bc=bc, U=None, recon=PLM, precision=prec,
                 block=_default_block((N, N, N)), name=typ, meta=dict(kind=typ, N=N, sub=sub))
    if generate:
        pb = pb.with_(U=generate_state(pb))
    return pb, steps


def generate_state(pb) -> np.ndarray:
    """Conserved state of a serving-stream problem built from its metadata."""
    kind, N, sub = pb.meta["kind"], pb.meta["N"], pb.meta["sub"]
    if kind == "sod":
        full = sod(N=N, seed=sub)
    elif kind == "kh":
        full = kelvin_helmholtz(N=N, seed=sub)
    else:
        full = sedov(N=N, seed=sub)
    assert full.n == tuple(pb.n) and full.bc == pb.bc and full.lo == pb.lo
    return full.U


# --------------------------------------------------------------------------
# Statically refined meshes (state layout only; no solver arithmetic)
# --------------------------------------------------------------------------
def to_leaves(U0, U1, leaves, block):
    """Leaf-major state [leaf][5][bz][by][bx] of a refined mesh: leaf
    (level, lx, ly, lz) takes block (lx, ly, lz) of the global state at its
    level, U0 [5][nz][ny][nx] for level 0 and U1 (twice the cells per axis)
    for level 1. ``leaves`` comes from the solver's leaf query."""
    bx, by, bz = (int(b) for b in block)
    lv = np.asarray(leaves).reshape(-1, 4)
    out = np.empty((len(lv), 5, bz, by, bx), dtype=np.float64)
    for q, (L, lx, ly, lz) in enumerate(lv):
        src = U0 if L == 0 else U1
        out[q] = src[:, lz * bz:(lz + 1) * bz, ly * by:(ly + 1) * by, lx * bx:(lx + 1) * bx]
    return out


def from_leaves(UL, leaves, block, level):
    """Inverse of ``to_leaves`` for one level: a dict {(lx, ly, lz): block}
    of that level's leaves."""
    lv = np.asarray(leaves).reshape(-1, 4)
    return {(int(r[1]), int(r[2]), int(r[3])): UL[q] for q, r in enumerate(lv) if r[0] == level}


def refine_boxes(refine):
    """The refined boxes of ``Problem.refine`` as a list of ((lo), (hi)) in
    root blocks: ``refine`` is one box or a sequence of boxes."""
    if refine is None:
        return []
    if len(refine) == 2 and all(np.isscalar(x) for x in refine[0]):
        return [(tuple(int(x) for x in refine[0]), tuple(int(x) for x in refine[1]))]
    return [(tuple(int(x) for x in b[0]), tuple(int(x) for x in b[1])) for b in refine]


def refined(make, refine, leaves):
    """A problem on a statically refined mesh. ``make(s)`` builds the uniform
    problem at s times the root resolution (s = 1, 2) on the same domain with
    the same block size; ``refine`` = ((lo), (hi)) in root blocks, or a
    sequence of such boxes; ``leaves`` fixes the leaf order. Each leaf's cells
    are sampled from the problem at its own resolution."""
    p1 = make(1)
    lv = np.asarray(leaves).reshape(-1, 4)
    p2 = make(2) if (lv[:, 0] == 1).any() else None
    UL = to_leaves(p1.U, None if p2 is None else p2.U, lv, p1.block)
    boxes = refine_boxes(refine)
    return p1.with_(U=UL, refine=boxes[0] if len(boxes) == 1 else tuple(boxes),
                    name=(p1.name + " refined").strip())
