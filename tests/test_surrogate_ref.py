"""Pins of the surrogate's CPU reference network (oracle/surrogate_ref.py):
brute-force loops for the periodic/zero-padded dilated convolution, exact
bfloat16 rounding cases, finite differences for its gradients; and the
surrogate library's exports."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ref():
    from oracle import surrogate_ref
    return surrogate_ref


def _brute_conv(x, w, b, d):
    cin, B, H, W = x.shape
    cout = w.shape[0]
    out = np.zeros((cout, B, H, W))
    for o in range(cout):
        for bb in range(B):
            for y in range(H):
                for j in range(W):
                    s = b[o]
                    for c in range(cin):
                        for ky in range(3):
                            for kx in range(3):
                                yy = y + d * (ky - 1)
                                if not 0 <= yy < H:
                                    continue
                                jj = (j + d * (kx - 1)) % W
                                s += w[o, c * 9 + ky * 3 + kx] * x[c, bb, yy, jj]
                    out[o, bb, y, j] = s
    return out


@pytest.mark.parametrize("d", [1, 2, 3])
def test_conv_matches_brute_force_loops(ref, d):
    rng = np.random.default_rng(3 + d)
    x = rng.standard_normal((2, 2, 5, 7))
    w = rng.standard_normal((3, 18))
    b = rng.standard_normal(3)
    assert np.allclose(ref.conv3x3(x, w, b, d), _brute_conv(x, w, b, d), atol=1e-12)


def test_bf16_rounding_cases(ref):
    import torch
    one = 1.0
    cases = {one: one, one + 2 ** -8: one, one + 3 * 2 ** -8: one + 2 ** -6, -2.5: -2.5,
             one + 2 ** -7: one + 2 ** -7, 3.0e-3 * (1 + 2 ** -10): None}
    for v, want in cases.items():
        got = ref.bf16_round(np.float32(v))
        if want is not None:
            assert got == want, (v, got, want)
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(10000) * 10.0 ** rng.integers(-4, 4, 10000)).astype(np.float32)
    lib = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ref.bf16_round(x), lib)


def test_backward_matches_central_differences(ref):
    rng = np.random.default_rng(11)
    layers = [(rng.standard_normal((3, 18)) * 0.4, rng.standard_normal(3) * 0.1, 3, 1, True),
              (rng.standard_normal((3, 27)) * 0.3, rng.standard_normal(3) * 0.1, 3, 2, True),
              (rng.standard_normal((2, 3)) * 0.5, rng.standard_normal(2) * 0.1, 1, 1, False)]
    x = rng.standard_normal((2, 1, 4, 6))
    dy = rng.standard_normal((2, 1, 4, 6))
    out, trace = ref.forward(x, layers, 0.1)
    grads, gx = ref.backward(dy, layers, trace, 0.1)

    def f(ls, xx):
        return float(np.sum(ref.forward(xx, ls, 0.1)[0] * dy))

    h = 1e-6
    for li, pick in [(0, (1, 5)), (1, (2, 20)), (2, (0, 2))]:
        w, b, k, d, a = layers[li]
        wp, wm = w.copy(), w.copy()
        wp[pick] += h
        wm[pick] -= h
        lp = list(layers)
        lm = list(layers)
        lp[li] = (wp, b, k, d, a)
        lm[li] = (wm, b, k, d, a)
        fd = (f(lp, x) - f(lm, x)) / (2 * h)
        assert abs(fd - grads[li][0][pick]) < 1e-6 * max(1.0, abs(fd))
    for pick in [(0, 0, 1, 2), (1, 0, 3, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[pick] += h
        xm[pick] -= h
        fd = (f(layers, xp) - f(layers, xm)) / (2 * h)
        assert abs(fd - gx[pick]) < 1e-6 * max(1.0, abs(fd))


def test_surrogate_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2501_07979_amd", "libzsur.so")
    if not os.path.exists(path):
        pytest.skip("libzsur.so not built")
    hdr = open(os.path.join(ROOT, "include", "zsur.h")).read()
    declared = sorted(set(re.findall(r"\b(zsur_[a-z0-9_]+)\s*\(", hdr)))
    lib = ctypes.CDLL(path)
    for name in declared:
        assert hasattr(lib, name), name
    from paper_2501_07979_amd import surrogate
    assert sorted(surrogate.EXPORTS) == declared
