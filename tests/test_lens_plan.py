"""Host logic of the lens helpers (no GPU): which zones count as narrow, the
device-memory estimate, the grouping of zones into waves and the memory a
design iteration adds per zone."""
import numpy as np

from paper_2501_07979_amd import lens
from paper_2501_07979_amd.workloads import Workload, c4, lwir_lens


def test_device_bytes_estimate_counts_fields_eps_layers_and_dft():
    w = Workload("z", r_in=100.0, nr=20, nphi=30, nz=40, n_fold=8, pml=(2, 3, 4, 5))
    cells, plane = 20 * 30 * 40, 20 * 30
    aux = (10 * 40 * 5 * 30 + 4 * 9 * plane) * 8
    assert lens.zone_device_bytes(w) == cells * (96 + 4) + 3 * aux + 8 * 2 * plane * 8
    assert lens.zone_device_bytes(w, both_sets=False) == cells * (48 + 4) + aux + 8 * 2 * plane * 8


def test_waves_respect_budget_family_and_cover_every_zone_once():
    zones = c4(12)
    ws = lwir_lens()[:3] + zones
    budget = 3 * max(lens.zone_device_bytes(w) for w in zones)
    waves = lens.plan_waves(ws, budget)
    seen = sorted(q for _, idx in waves for q in idx)
    assert seen == list(range(len(ws)))
    for fam, idx in waves:
        narrow = {lens.is_narrow(ws[q]) for q in idx}
        assert len(narrow) == 1 and fam == (lens.FLAT if narrow.pop() else lens.TWO_STEP)
        if len(idx) > 1:
            assert sum(lens.zone_device_bytes(ws[q]) for q in idx) <= budget
    # with one launch for all, the order is kept and only the budget cuts
    waves = lens.plan_waves(ws, budget, tile_rows=32)
    assert [q for _, idx in waves for q in idx] == list(range(len(ws)))
    assert all(f == 32 for f, _ in waves)


def test_waves_with_given_sizes_and_iteration_reserve():
    """Waves planned on given per-zone sizes (the exact time-stepping bytes a
    zone reports) cut on those sizes; the bytes a design iteration adds per
    zone are the forward and adjoint design-volume DFTs, the adjoint source
    and the iteration's tensors."""
    ws = c4(12)
    sizes = [1000 + 10 * q for q in range(len(ws))]
    budget = 3500
    waves = lens.plan_waves(ws, budget, sizes=sizes)
    assert sorted(q for _, idx in waves for q in idx) == list(range(len(ws)))
    for _, idx in waves:
        assert len(idx) == 1 or sum(sizes[q] for q in idx) <= budget
    assert [len(idx) for _, idx in waves] == [3, 3, 3, 3]
    # a budget below every zone: one zone per wave
    assert [len(idx) for _, idx in lens.plan_waves(ws, 1, sizes=sizes)] == [1] * len(ws)
    w = ws[0]
    K, plane, nd = len(w.omegas), w.nr * w.nphi, w.design[1] - w.design[0]
    assert lens.iteration_bytes(w) == 2 * K * 3 * nd * plane * 8 + 6 * K * 2 * plane * 8 + 2 * nd * plane * 4


def test_lwir_lens_geometry():
    ws = lwir_lens()
    assert len(ws) == 16 and ws[0].n_fold == 0 and ws[0].axis == 1 and ws[0].nphi == 1
    for l, w in enumerate(ws[1:], start=2):
        assert w.n_fold == 720 * l and w.nr == 1250
        r_out = w.r_in + w.nr
        assert r_out * 2 * np.pi / (w.n_fold * w.nphi) <= 0.021 * 50 + 1e-9    # r dphi <= 0.021 lambda
        assert lens.is_narrow(w)
