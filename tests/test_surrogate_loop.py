"""Host logic of the surrogate-assisted design loop (CPU, no GPU): the FDTD
re-check is the arbiter and the fallback.  With an analytic objective standing
in for the FDTD-adjoint evaluation: a surrogate whose gradient is right
speeds the ascent; a corrupted surrogate (its weights scrambled: a gradient
pointing away from the optimum, or non-finite values) has every block of its
steps rejected, and the accepted patterns are exactly those of plain
FDTD-adjoint ascent."""
import numpy as np
import torch

from paper_2501_07979_amd.surrogate import adam_update, checked_loop

N = 64
TARGET = torch.tensor(np.random.default_rng(1).uniform(0.2, 0.8, N), dtype=torch.float64)


def fdtd(rho):
    d = rho - TARGET
    return float(-(d * d).sum()), -2.0 * d


def plain(rho0, steps, lr):
    rho = rho0.clone()
    m, v = torch.zeros_like(rho), torch.zeros_like(rho)
    seq = [rho.clone()]
    for t in range(1, steps + 1):
        _, g = fdtd(rho)
        adam_update(rho, g, m, v, t, lr)
        seq.append(rho.clone())
    return seq


def test_good_surrogate_is_accepted_and_speeds_the_ascent():
    rho0 = torch.full((N,), 0.5, dtype=torch.float64)
    _, F_sur, hist = checked_loop(fdtd, lambda r: fdtd(r)[1] * 1.05, rho0, outer=6, inner=9, lr=0.01)
    F_plain = fdtd(plain(rho0, 6, 0.01)[-1])[0]
    assert all(h["accepted"] for h in hist)
    assert F_sur > F_plain


def _corrupted_run(sur):
    rho0 = torch.full((N,), 0.5, dtype=torch.float64)
    seen = []
    best, F, hist = checked_loop(lambda r: (seen.append(r.clone()), fdtd(r))[1], sur, rho0, outer=12, inner=5,
                                 lr=0.01)
    return rho0, seen, best, F, hist


def test_corrupted_surrogate_is_rejected_and_falls_back_to_plain_steps():
    for sur in (lambda r: -50.0 * fdtd(r)[1],                       # scrambled: uphill is downhill
                lambda r: torch.full_like(r, float("nan"))):          # non-finite weights
        rho0, seen, best, F, hist = _corrupted_run(sur)
        blocks = [h for h in hist if h["surrogate_block"]]
        assert blocks and not any(h["accepted"] for h in blocks)
        accepted = [seen[q] for q, h in enumerate(hist) if h["accepted"]]
        ref = plain(rho0, len(accepted) - 1, 0.01)
        for a, b in zip(accepted, ref):
            assert torch.equal(a, b)
        assert torch.isfinite(best).all() and F == fdtd(best)[0]
        # the accepted objective never falls
        Fs = [h["F_fdtd"] for h in hist if h["accepted"]]
        assert all(b >= a for a, b in zip(Fs, Fs[1:]))
