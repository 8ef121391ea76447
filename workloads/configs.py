"""Workload definitions: plain data and seeded primitive fields.

Physical set-up (Sec. 3.1 of arXiv:1705.04374, with the constants of the
synthetic clouds used here): water/air stiffened gases, air bubbles at low
pressure inside a cloud, a smooth pressure ramp to the ambient pressure just
outside the cloud, fluid at rest, unit domain with the cloud at its centre.

Cloud distributions (the paper's: positions uniform in the cloud, log-normal
radii, Sec. 3 and 3.1):
  cloud2d   2-D, 8 discs in a disk of radius 0.3, radii LogN(median 0.03, sigma 0.25)
  cloud50   3-D, 50 bubbles in a ball of radius 0.25, radii LogN(0.02, 0.3)
  cloud500  3-D, 500 bubbles in a ball of radius 0.3, radii LogN(0.015, 0.1)
            clipped to [0.8, 1.2] x median (the paper's shape: cloud radius
            20 bubble radii, radii clipped to +-20 %)
Bubbles never overlap (rejection).
"""
from __future__ import annotations

import math

import numpy as np

MASTER_SEED = 170504374

EOS = dict(gamma1=6.12, pc1=3.43e8, gamma2=1.4, pc2=0.0)

BASE = dict(
    eos=EOS,
    rho1=1000.0,        # water density [kg/m^3]
    rho2=1.0,           # air density
    p_bubble=2340.0,    # 0.0234 bar inside the cloud
    p_inf=1.0e7,        # 100 bar ambient
    cfl=0.3,
    n_sub=4,            # sub-samples per axis for the initial volume fraction
    weno_eps=1e-6,
    bc="zero_gradient",
    center=(0.5, 0.5, 0.5),
)

CLOUDS = {
    "cloud2d": dict(ndim=2, n_bubbles=8, cloud_radius=0.3, r_median=0.03, r_sigma=0.25,
                    r_lo=0.0, r_hi=0.0),
    "cloud50": dict(ndim=3, n_bubbles=50, cloud_radius=0.25, r_median=0.02, r_sigma=0.3,
                    r_lo=0.0, r_hi=0.0),
    "cloud500": dict(ndim=3, n_bubbles=500, cloud_radius=0.3, r_median=0.015, r_sigma=0.1,
                     r_lo=0.8 * 0.015, r_hi=1.2 * 0.015),
}

# End time: f_T Rayleigh collapse times of a median bubble under the ambient
# over-pressure (t_R = 0.915 R sqrt(rho / dp), Rayleigh 1917).  The paper
# simulates about 70 us for 1 mm bubbles, 7.5 such times.
F_T = 7.5


def rayleigh_time(cloud: str) -> float:
    c = CLOUDS[cloud]
    return 0.915 * c["r_median"] * math.sqrt(BASE["rho1"] / (BASE["p_inf"] - BASE["p_bubble"]))


def t_end(cloud: str) -> float:
    return F_T * rayleigh_time(cloud)


def solver_config(cloud: str, n: int, **over) -> dict:
    """Plain dict describing one solve of a cloud at n cells per side."""
    c = CLOUDS[cloud]
    cfg = dict(BASE)
    cfg.update(ndim=c["ndim"], n=n, cloud=cloud, cloud_radius=c["cloud_radius"],
               ramp_delta=c["cloud_radius"] / 20.0, ramp_width=c["cloud_radius"] / 3.0)
    cfg.update(over)
    return cfg


def cloud_spec(cloud: str) -> dict:
    c = dict(CLOUDS[cloud])
    c["center"] = BASE["center"]
    return c


# The five workloads, in the order the benchmark description lists them.
WORKLOADS = {
    "cloud2d_mlmc": dict(cloud="cloud2d", levels=[32, 64], samples=[16, 4], precision="f64",
                         t_end=t_end("cloud2d")),
    "single3d_128": dict(cloud="cloud50", n=128, steps=200, precision=("f64", "f32")),
    "single3d_256": dict(cloud="cloud500", n=256, steps=200, precision=("f32", "f64")),
    "batched3": dict(cloud="cloud500", levels=[64, 128, 256], samples=[256, 48, 8],
                     precision="f32", t_end=t_end("cloud500")),
    "learned": dict(cloud="cloud500", n=64, train_samples=4096, eval_sets=65536),
    "full_ofmlmc": dict(cloud="cloud500", levels=[64, 128, 256, 512], precision="f32",
                        rel_tol=0.01, t_end=t_end("cloud500")),
}

# ---------------------------------------------------------------------------
# Neutral primitive fields for the solver tests (plain arrays; the conversion
# to conserved variables is done by each side with its own EOS code).
# Layout: [nv, nz, ny, nx] with nv = 4 + ndim, slots
# (a1r1, a2r2, u_1..u_d, p, a2).
# ---------------------------------------------------------------------------


def _grid_shape(ndim: int, n: int):
    return (n if ndim > 2 else 1, n if ndim > 1 else 1, n)


def riemann_primitives(ndim: int, n: int, left: dict, right: dict, x0: float = 0.5,
                       axis: int = 0) -> np.ndarray:
    """Piecewise-constant primitive state split at x0 along `axis`.
    left/right: dict(a1r1, a2r2, u, p, a2) with u the velocity along `axis`."""
    nz, ny, nx = _grid_shape(ndim, n)
    W = np.zeros((4 + ndim, nz, ny, nx))
    idx = np.arange(n)
    xc = (idx + 0.5) / n
    mask = xc < x0
    shape = [1, 1, 1]
    shape[2 - axis] = n
    m = mask.reshape(shape)
    for slot, key in ((0, "a1r1"), (1, "a2r2"), (2 + ndim, "p"), (3 + ndim, "a2")):
        W[slot] = np.where(m, left[key], right[key])
    W[2 + axis] = np.where(m, left.get("u", 0.0), right.get("u", 0.0))
    return W


def random_smooth_primitives(ndim: int, n: int, seed: int, rho1=1000.0, rho2=1.0,
                             p_mean=1.0e6, p_amp=2.0e5, u_amp=20.0, a2_amp=0.3) -> np.ndarray:
    """Smooth periodic random primitive state (a few Fourier modes per field)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = _grid_shape(ndim, n)
    zz, yy, xx = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    coords = [xx, yy, zz]

    def field():
        f = np.zeros_like(xx)
        for _ in range(3):
            kv = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            arg = sum(2 * np.pi * kv[a] * coords[a] for a in range(ndim))
            f += np.cos(arg + ph) / 3.0
        return f

    W = np.zeros((4 + ndim, nz, ny, nx))
    a2 = 0.5 + a2_amp * field()
    W[3 + ndim] = a2
    W[0] = (1.0 - a2) * rho1 * (1.0 + 0.05 * field())
    W[1] = a2 * rho2 * (1.0 + 0.05 * field())
    for m in range(ndim):
        W[2 + m] = u_amp * field()
    W[2 + ndim] = p_mean + p_amp * field()
    return W


def interface_primitives(ndim: int, n: int, seed: int, u=(35.0, -20.0, 10.0), p=1.0e5,
                         rho1=1000.0, rho2=1.0) -> np.ndarray:
    """Uniform velocity and pressure; a2 jumps between 0 and 1 on random
    blocks, so phase densities and the mixture jump sharply."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = _grid_shape(ndim, n)
    blocks = max(n // 8, 1)
    coarse = rng.integers(0, 2, size=(max(nz // 8, 1), max(ny // 8, 1), blocks)).astype(np.float64)
    a2 = np.kron(coarse, np.ones((min(8, nz), min(8, ny), 8)))[:nz, :ny, :nx]
    W = np.zeros((4 + ndim, nz, ny, nx))
    W[3 + ndim] = a2
    W[0] = (1.0 - a2) * rho1
    W[1] = a2 * rho2
    for m in range(ndim):
        W[2 + m] = u[m]
    W[2 + ndim] = p
    return W
