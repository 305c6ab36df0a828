"""Seeded request trace for the served stream: Poisson arrivals, each
request a disk of the full-size config family with mixed cube sizes."""
from __future__ import annotations

import numpy as np


def make_trace(rate_hz: float = 200.0, duration_s: float = 60.0, seed: int = 5,
               pix=(64, 128, 256, 512), chans=(16, 32, 64, 128), samp=(128, 512),
               grad_frac: float = 0.25, max_requests=None):
    """List of dicts: t_arrive [s], nx=ny, nch, nsamp, grad (bool), disk_seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        n = int(rng.choice(pix))
        out.append(dict(t_arrive=t, nx=n, ny=n, nch=int(rng.choice(chans)),
                        nsamp=int(rng.integers(samp[0], samp[1] + 1)),
                        grad=bool(rng.random() < grad_frac),
                        disk_seed=int(rng.integers(0, 2 ** 31 - 1))))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out
