"""Oracle of the random cloud geometry omega (Sec. 3 and 3.1 of arXiv:1705.04374).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

The paper draws bubble centres uniformly inside the cloud and radii from a
log-normal law, clipped to a range (Sec. 3.1; 500 bubbles give 2000 random
dimensions).  This module is an independent pure-Python implementation of the
same draw as the library's host sampler; both are written from these
definitions:

  generator  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state
             advances by 0x9E3779B97F4A7C15 and each output is the state
             passed through the mixer
             z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
             z *= 0x94D049BB133111EB; z ^= z>>31.
  stream     the initial state for (seed, term, index) is
             mix(mix(mix(seed) ^ term) ^ index), with mix(x) the first output
             of a generator whose state is x.
  uniform    U = (x >> 11) * 2^-53 in [0, 1).
  centre     draw v in [-1,1]^d coordinate by coordinate until |v|^2 < 1;
             centre = cloud centre + R v.
  radius     Box-Muller: u1 = 1 - U, u2 = U, Z = sqrt(-2 ln u1) cos(2 pi u2);
             r = median exp(sigma Z), redrawn while outside [r_lo, r_hi] when
             a range is given.
  overlap    a candidate overlapping an accepted bubble,
             |c - c_j|^2 < (r + r_j)^2, is discarded with its radius and a new
             centre and radius are drawn; at most 100000 candidates per bubble.
"""
from __future__ import annotations

import math

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MAX_TRIES = 100000


def _mix_output(state: int) -> int:
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def mix(x: int) -> int:
    """First output of a SplitMix64 generator whose state is x."""
    return _mix_output((x + GOLDEN) & MASK)


class SplitMix64:
    def __init__(self, state: int):
        self.state = state & MASK

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & MASK
        return _mix_output(self.state)

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def stream(seed: int, term: int, index: int) -> SplitMix64:
    return SplitMix64(mix(mix(mix(seed & MASK) ^ (term & MASK)) ^ (index & MASK)))


class Infeasible(RuntimeError):
    pass


def sample_cloud(spec: dict, seed: int, term: int, index: int) -> np.ndarray:
    """Bubbles (n_b x 4: x, y, z, r) of the cloud omega(seed, term, index)."""
    d = spec["ndim"]
    nb = spec["n_bubbles"]
    R = spec["cloud_radius"]
    cen = spec.get("center", (0.5, 0.5, 0.5))
    med, sig = spec["r_median"], spec["r_sigma"]
    lo, hi = spec.get("r_lo", 0.0), spec.get("r_hi", 0.0)
    clip = hi > 0.0
    g = stream(seed, term, index)
    out = np.zeros((nb, 4))
    for b in range(nb):
        tries = 0
        while True:
            tries += 1
            if tries > MAX_TRIES:
                raise Infeasible("bubble %d: no non-overlapping position after %d tries" % (b, MAX_TRIES))
            while True:
                v = [2.0 * g.uniform() - 1.0 for _ in range(d)]
                n2 = v[0] * v[0]
                for a in range(1, d):
                    n2 = n2 + v[a] * v[a]
                if n2 < 1.0:
                    break
            c = [cen[a] + R * v[a] for a in range(d)] + [0.0] * (3 - d)
            while True:
                u1 = 1.0 - g.uniform()
                u2 = g.uniform()
                z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
                r = med * math.exp(sig * z)
                if not clip or (lo <= r <= hi):
                    break
            ok = True
            for j in range(b):
                dx = c[0] - out[j, 0]
                d2 = dx * dx
                for a in range(1, d):
                    da = c[a] - out[j, a]
                    d2 = d2 + da * da
                s = r + out[j, 3]
                if d2 < s * s:
                    ok = False
                    break
            if ok:
                out[b, :3] = c
                out[b, 3] = r
                break
    return out
