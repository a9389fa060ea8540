"""Seeded random refined-mesh configurations shared by the reference-solver
pins and the GPU parity tests (inputs only: no solver arithmetic here)."""
import numpy as np

from paper_2409_16053_amd import problems as P


def smooth(n, bc, seed, block, **kw):
    """Smooth seeded fields on an n-cell unit box (cell-centre values):
    density, velocity and pressure from a few low Fourier modes."""
    rng = np.random.default_rng(seed)
    c = [(np.arange(n[d]) + 0.5) / n[d] for d in range(3)]
    z, y, x = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, size=8)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * y + ph[1])
    vx = 0.4 * np.sin(2 * np.pi * (y + z) + ph[2])
    vy = 0.3 * np.cos(2 * np.pi * (x - z) + ph[3])
    vz = 0.2 * np.sin(2 * np.pi * (x + y) + ph[4])
    p = 1.0 + 0.2 * np.cos(2 * np.pi * z + ph[5]) * np.sin(2 * np.pi * x + ph[6])
    pb = P.uniform(n=tuple(n), rho=1.0, v=(0, 0, 0), p=1.0)
    return pb.with_(U=P.conserved(rho, vx, vy, vz, p, pb.gamma), bc=bc, block=block, **kw)


def random_config(seed):
    """(recon, rk, root cells n, block, refined box lo, hi, boundaries) drawn
    from seed 1000 + seed."""
    rng = np.random.default_rng(1000 + seed)
    recon = int(rng.choice([P.PLM, P.PPM4, P.WENOZ, P.PPMX]))
    rk = int(rng.integers(1, 5))
    int(rng.choice([P.FP64, P.MIXED]))  # (kept so that the later draws stay put)
    nr = rng.integers(2, 4, size=3)
    block = tuple(int(b) for b in rng.choice([8, 12, 16], size=3))
    n = tuple(int(nr[d] * block[d]) for d in range(3))
    lo = tuple(int(rng.integers(0, nr[d])) for d in range(3))
    hi = tuple(int(rng.integers(lo[d] + 1, nr[d] + 1)) for d in range(3))
    bc = tuple((b, b) for b in rng.choice([P.PERIODIC, P.OUTFLOW], size=3))
    return recon, rk, n, block, lo, hi, bc


def random_refined(seed, leaves, recon=None):
    """The refined problem of ``random_config(seed)`` (``recon`` overrides the
    drawn reconstruction); ``leaves(pb)`` gives a refined problem's leaf table."""
    r, rk, n, block, lo, hi, bc = random_config(seed)
    recon = r if recon is None else recon
    make = lambda s: smooth([n[d] * s for d in range(3)], bc, seed, block, recon=recon, rk=rk)
    base = make(1).with_(refine=(lo, hi))
    return P.refined(make, (lo, hi), leaves(base))


def one_ulp_sensitivity(advance, pb, steps):
    """Relative L1 change of a solver's result when half of the initial values
    (a seeded choice) move up by one ulp: how far apart two correct FP64
    implementations, differing by rounding only, can be expected to end."""
    r0 = advance(pb, steps)
    U1 = pb.U.copy()
    mask = np.random.default_rng(1).random(U1.shape) < 0.5
    U1[mask] = np.nextafter(U1[mask], np.inf)
    r1 = advance(pb, steps, U=U1)
    return float(np.abs(r1["U"] - r0["U"]).sum() / np.abs(r0["U"]).sum())
