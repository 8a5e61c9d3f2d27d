"""Host logic of the two-step launch plan (no GPU): the tiles own every cell
of the zone exactly once; the interior tiles compute no layer cell (their
rows i0-2 .. i0+rows and planes kb-2 .. ke, clipped to the zone, avoid both
layers), so they may run the instantiation without layer recursions; the
owned columns of interior tiles start on 64 B boundaries; every tile order
is a permutation of the natural one.  The flat-mapped two-step plan (launch
code 34) gives every tile all phi cells and at most 256 / nphi - 3 rows, and
its z-layer-only tiles (kind 2) compute no r-layer row."""
import numpy as np
import pytest

ZONES = {
    "production_like": dict(nr=64, nphi=128, nz=60, pml=(12, 12, 12, 12)),
    "ragged": dict(nr=37, nphi=130, nz=41, pml=(5, 6, 4, 7)),
    "no_layers": dict(nr=29, nphi=64, nz=33, pml=(0, 0, 0, 0)),
    "axis_zone": dict(nr=45, nphi=1, nz=50, pml=(0, 6, 4, 7)),
    "thin": dict(nr=3, nphi=5, nz=4, pml=(1, 1, 1, 1)),
    "layers_8": dict(nr=48, nphi=96, nz=40, pml=(8, 8, 8, 8)),
}


def _desc(zda, nr, nphi, nz, pml):
    return zda.default_desc(r_in=1000.0, nr=nr, nphi=nphi, nz=nz, n_fold=8, m=1, pml=pml, k_mon=nz - 2,
                            design=(1, 2))


@pytest.mark.parametrize("tile_rows", [5, 13])
@pytest.mark.parametrize("kchunk", [3, 9, 48])
@pytest.mark.parametrize("name", list(ZONES))
def test_tiles_cover_each_cell_once(name, kchunk, tile_rows):
    from paper_2501_07979_amd import zda
    z = ZONES[name]
    d = _desc(zda, **z)
    tiles, n_int = zda.plan_two_step_tiles(d, tile_rows, kchunk, k_src=2)
    nr, nphi, nz = z["nr"], z["nphi"], z["nz"]
    pr0, pr1, pz0, pz1 = z["pml"]
    own = np.zeros((nz, nr, nphi), np.int32)
    for q, (bx, y, zz, kind) in enumerate(tiles):
        i0, rows = int(y & 0xFFFF), int(y >> 16)
        kb, ke = int(zz & 0xFFFF), int(zz >> 16)
        cols = 56 if kind == 0 else 61
        assert (kind == 0) == (q < n_int)
        assert 1 <= rows <= tile_rows and kb < ke
        j0 = int(bx) * cols
        assert j0 < nphi
        own[kb:ke, i0:i0 + rows, j0:min(j0 + cols, nphi)] += 1
        if kind == 0:
            assert (j0 * 8) % 64 == 0
            r_lo, r_hi = max(i0 - 2, 0), min(i0 + rows, nr - 1)
            k_lo, k_hi = max(kb - 2, 0), min(ke, nz - 1)
            assert pr0 <= r_lo and r_hi < nr - pr1, (i0, rows)
            assert pz0 <= k_lo and k_hi < nz - pz1, (kb, ke)
    assert own.min() == 1 and own.max() == 1


@pytest.mark.parametrize("order", [1, (4 << 8) | 8, (1 << 8) | 3, (2 << 8) | 1])
def test_tile_orders_are_permutations(order):
    from paper_2501_07979_amd import zda
    for z in ZONES.values():
        d = _desc(zda, **z)
        base, n0 = zda.plan_two_step_tiles(d, 13, 9, k_src=2)
        other, n1 = zda.plan_two_step_tiles(d, 13, 9, k_src=2, order=order)
        assert n0 == n1
        for part in (slice(0, n0), slice(n0, None)):
            a = sorted(map(tuple, base[part].tolist()))
            b = sorted(map(tuple, other[part].tolist()))
            assert a == b


def test_plan_rejects_bad_arguments():
    from paper_2501_07979_amd import zda
    d = _desc(zda, **ZONES["ragged"])
    for tr, kc, order in [(7, 9, 0), (13, 0, 0), (13, 9, (0 << 8) | 4)]:
        with pytest.raises(zda.ZdaError) as e:
            zda.plan_two_step_tiles(d, tr, kc, order=order)
        assert e.value.status == zda.ZDA_ERR_ARG


NARROW = {
    "continuous_axis": dict(nr=300, nphi=1, nz=41, pml=(0, 6, 4, 7)),
    "wedge11": dict(nr=1250, nphi=11, nz=60, pml=(12, 12, 10, 10)),
    "wedge16_ragged": dict(nr=37, nphi=16, nz=33, pml=(5, 6, 4, 7)),
    "wedge32": dict(nr=29, nphi=32, nz=20, pml=(3, 3, 3, 3)),
    "thin": dict(nr=3, nphi=5, nz=4, pml=(1, 1, 1, 1)),
}


@pytest.mark.parametrize("kchunk", [3, 16])
@pytest.mark.parametrize("name", list(NARROW))
def test_flat_two_step_tiles(name, kchunk):
    from paper_2501_07979_amd import zda
    z = NARROW[name]
    d = _desc(zda, **z)
    tiles, n_int = zda.plan_two_step_tiles(d, 34, kchunk, k_src=2)
    nr, nphi, nz = z["nr"], z["nphi"], z["nz"]
    pr0, pr1, pz0, pz1 = z["pml"]
    rows_max = 256 // nphi - 3
    own = np.zeros((nz, nr), np.int32)
    for q, (bx, y, zz, kind) in enumerate(tiles):
        i0, rows = int(y & 0xFFFF), int(y >> 16)
        kb, ke = int(zz & 0xFFFF), int(zz >> 16)
        assert bx == 0 and (kind == 0) == (q < n_int) and kind in (0, 2, 3)
        assert 1 <= rows <= rows_max and kb < ke and ke - kb <= kchunk
        own[kb:ke, i0:i0 + rows] += 1
        if kind == 2:           # z-layer recursions only: no computed row in an r-layer
            r_lo, r_hi = max(i0 - 2, 0), min(i0 + rows, nr - 1)
            assert pr0 <= r_lo and r_hi < nr - pr1, (i0, rows)
        if kind == 0:
            r_lo, r_hi = max(i0 - 2, 0), min(i0 + rows, nr - 1)
            k_lo, k_hi = max(kb - 2, 0), min(ke, nz - 1)
            assert pr0 <= r_lo and r_hi < nr - pr1, (i0, rows)
            assert pz0 <= k_lo and k_hi < nz - pz1, (kb, ke)
    assert own.min() == 1 and own.max() == 1


def test_flat_two_step_plan_refuses_wide_zones():
    from paper_2501_07979_amd import zda
    d = _desc(zda, nr=20, nphi=33, nz=20, pml=(3, 3, 3, 3))
    with pytest.raises(zda.ZdaError) as e:
        zda.plan_two_step_tiles(d, 34, 8)
    assert e.value.status == zda.ZDA_ERR_ARG


PLAN_CARRY = 1 << 16


@pytest.mark.parametrize("tile_rows", [5, 13])
@pytest.mark.parametrize("kchunk", [3, 48])
@pytest.mark.parametrize("name", list(ZONES))
def test_carry_plan_tiles(name, kchunk, tile_rows):
    """The plan of ZDA_OPT_LAYER_CARRY: every cell owned once; kind 1 tiles
    (r-layer rows, auxiliaries carried in registers) own at most 5 rows;
    kind 4 tiles (r-layer rows, r-layer recursions only) own at most 7 rows
    and compute no z-layer plane, and a band holds them only where 7-row
    tiles take fewer wavefront rows (10 per tile) than 5-row ones (8 per
    tile); kind 2 tiles compute no r-layer row; the interior tiles are those
    of the plain plan."""
    from paper_2501_07979_amd import zda
    z = ZONES[name]
    d = _desc(zda, **z)
    tiles, n_int = zda.plan_two_step_tiles(d, tile_rows, kchunk, k_src=2, order=PLAN_CARRY)
    plain, n_plain = zda.plan_two_step_tiles(d, tile_rows, kchunk, k_src=2)
    assert n_int == n_plain
    assert sorted(map(tuple, tiles[:n_int].tolist())) == sorted(map(tuple, plain[:n_plain].tolist()))
    nr, nphi, nz = z["nr"], z["nphi"], z["nz"]
    pr0, pr1, pz0, pz1 = z["pml"]
    own = np.zeros((nz, nr, nphi), np.int32)
    for q, (bx, y, zz, kind) in enumerate(tiles):
        i0, rows = int(y & 0xFFFF), int(y >> 16)
        kb, ke = int(zz & 0xFFFF), int(zz >> 16)
        assert (kind == 0) == (q < n_int) and kind in (0, 1, 2, 4)
        cols = 56 if kind == 0 else 61
        assert 1 <= rows <= {1: 5, 4: 7}.get(int(kind), tile_rows) and kb < ke
        j0 = int(bx) * cols
        assert j0 < nphi
        own[kb:ke, i0:i0 + rows, j0:min(j0 + cols, nphi)] += 1
        r_lo, r_hi = max(i0 - 2, 0), min(i0 + rows, nr - 1)
        if kind == 2:
            assert pr0 <= r_lo and r_hi < nr - pr1, (i0, rows)
        if kind in (1, 4):
            assert r_lo < pr0 or r_hi >= nr - pr1, (i0, rows)
        if kind == 4:
            k_lo, k_hi = max(kb - 2, 0), min(ke, nz - 1)
            assert pz0 <= k_lo and k_hi < nz - pz1, (kb, ke)
            h = pr0 + 2 if i0 < pr0 + 2 else nr - (nr - pr1 - 1)
            assert -(-h // 7) * 10 < -(-h // 5) * 8, h
    assert own.min() == 1 and own.max() == 1


@pytest.mark.parametrize("kchunk", [3, 9, 48])
@pytest.mark.parametrize("name", list(ZONES))
def test_three_step_tiles_cover_each_cell_once(name, kchunk):
    """The three-step plan (tile_rows 11): every cell owned once; interior
    tiles (kind 0) own at most 11 rows and 56 phi cells starting on 64 B
    boundaries, and their computed rows i0-3 .. i0+rows+1 and planes kb-3 ..
    ke+1 hold no layer cell; kind 2 tiles (z-layer recursions only) compute
    no r-layer row; kind 3 tiles (r-layer bands) own at most 7 rows; layer
    tiles own 59 phi cells."""
    from paper_2501_07979_amd import zda
    z = ZONES[name]
    d = _desc(zda, **z)
    tiles, n_int = zda.plan_two_step_tiles(d, 11, kchunk, k_src=2)
    nr, nphi, nz = z["nr"], z["nphi"], z["nz"]
    pr0, pr1, pz0, pz1 = z["pml"]
    own = np.zeros((nz, nr, nphi), np.int32)
    for q, (bx, y, zz, kind) in enumerate(tiles):
        i0, rows = int(y & 0xFFFF), int(y >> 16)
        kb, ke = int(zz & 0xFFFF), int(zz >> 16)
        assert kind in (0, 2, 3) and (kind == 0) == (q < n_int)
        assert 1 <= rows <= (7 if kind == 3 else 11) and kb < ke
        cols = 56 if kind == 0 else 59
        j0 = int(bx) * cols
        assert j0 < nphi
        own[kb:ke, i0:i0 + rows, j0:min(j0 + cols, nphi)] += 1
        r_lo, r_hi = max(i0 - 3, 0), min(i0 + rows + 1, nr - 1)
        if kind in (0, 2):
            assert pr0 <= r_lo and r_hi < nr - pr1, (i0, rows)
        if kind == 0:
            assert (j0 * 8) % 64 == 0
            k_lo, k_hi = max(kb - 3, 0), min(ke + 1, nz - 1)
            assert pz0 <= k_lo and k_hi < nz - pz1, (kb, ke)
    assert own.min() == 1 and own.max() == 1
