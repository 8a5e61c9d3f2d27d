"""GPU tests of the design surrogate's kernels against the FP64 reference
network (oracle/surrogate_ref.py).  Tolerances follow the arithmetic: bf16
operands are exact inputs to FP32 accumulation, so a contraction over K terms
differs from the FP64 sum of the same bf16 values by ~sqrt(K) FP32 ulps
(<= 1e-5 relative here); gradients take dZ rounded to bf16 (unit roundoff
2^-9) where the reference keeps it exact, <= 1e-2 relative L2."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-surrogate]", *a, flush=True)


@pytest.fixture(scope="module")
def sur():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_07979_amd import surrogate as S
    S.load()
    return S


def _bf16_bits(vals):
    from oracle.surrogate_ref import bf16_round
    r = bf16_round(np.asarray(vals, np.float32)).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16), r.astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("dims", [(70, 130, 100), (72, 136, 104)])   # element-wise / 16 B tile loads
@pytest.mark.parametrize("a_rowmajor", [True, False])
@pytest.mark.parametrize("b_rowmajor", [True, False])
@pytest.mark.parametrize("split", [1, 3])
def test_gemm_every_layout_matches_fp64(sur, a_rowmajor, b_rowmajor, split, dims):
    import torch
    from oracle.surrogate_ref import bf16_round
    M, N, K = dims
    rng = np.random.default_rng(7 + 2 * a_rowmajor + b_rowmajor + 5 * split)
    a_bits, a_val = _bf16_bits(rng.standard_normal((M, K)))
    b_bits, b_val = _bf16_bits(rng.standard_normal((K, N)))
    if a_rowmajor:
        A, sam, sak = a_bits, K, 1
    else:
        A, sam, sak = np.ascontiguousarray(a_bits.T), 1, M
    if b_rowmajor:
        B, sbk, sbn = b_bits, N, 1
    else:
        B, sbk, sbn = np.ascontiguousarray(b_bits.T), 1, K
    bias = rng.standard_normal(M).astype(np.float32)
    dA = torch.tensor(A.view(np.int16), device="cuda")
    dB = torch.tensor(B.view(np.int16), device="cuda")
    dbias = torch.tensor(bias, device="cuda")
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    Cb = torch.zeros((M, N), dtype=torch.int16, device="cuda")
    work = torch.zeros(split * M * N, dtype=torch.float32, device="cuda")
    _say("gemm", a_rowmajor, b_rowmajor, split)
    sur._ck(sur.load().zsur_gemm(M, N, K, sur._p(dA), sam, sak, sur._p(dB), sbk, sbn, sur._p(C), N, sur._p(Cb),
                                 sur._p(dbias), sur.ACT_LEAKY, 0.1, split, sur._p(work), sur._stream()))
    z = a_val @ b_val + bias[:, None].astype(np.float64)
    ref = np.where(z > 0, z, 0.1 * z)
    got = C.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    cb = Cb.cpu().numpy().view(np.uint16)
    assert np.array_equal(cb, (bf16_round(got.astype(np.float32)).astype(np.float32).view(np.uint32) >> 16))


@pytest.mark.parametrize("dil", [1, 2, 3])
def test_im2col_gemm_is_the_reference_convolution(sur, dil):
    import torch
    from oracle import surrogate_ref as R
    rng = np.random.default_rng(20 + dil)
    cin, cout, B, H, W = 5, 7, 2, 9, 11
    x = rng.standard_normal((cin, B, H, W)).astype(np.float32)
    w = rng.standard_normal((cout, cin * 9)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    lib = sur.load()
    N = B * H * W
    dx = torch.tensor(x, device="cuda")
    cols = torch.empty((cin * 9, N), dtype=torch.int16, device="cuda")
    sur._ck(lib.zsur_im2col(sur._p(dx), cin, B, H, W, dil, sur._p(cols), sur._stream()))
    wb = torch.tensor(_bf16_bits(w)[0].view(np.int16), device="cuda")
    y = torch.empty((cout, N), dtype=torch.float32, device="cuda")
    sur._ck(lib.zsur_gemm(cout, N, cin * 9, sur._p(wb), cin * 9, 1, sur._p(cols), N, 1, sur._p(y), N, None,
                          sur._p(torch.tensor(b, device="cuda")), sur.ACT_NONE, 1.0, 1, None, sur._stream()))
    ref = R.conv3x3(R.bf16_round(x), R.bf16_round(w), b, dil)
    assert _rel(y.cpu().numpy().reshape(ref.shape), ref) <= 1e-6
    # col2im is the adjoint of im2col: <im2col(x), c> = <x, col2im(c)>
    c = rng.standard_normal((cin * 9, N)).astype(np.float32)
    out = torch.empty((cin, B, H, W), dtype=torch.float32, device="cuda")
    sur._ck(lib.zsur_col2im(sur._p(torch.tensor(c, device="cuda")), cin, B, H, W, dil, sur._p(out), sur._stream()))
    cols_v = (cols.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    lhs = float(np.sum(cols_v * c))
    rhs = float(np.sum(R.bf16_round(x) * out.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-5 * np.sum(np.abs(cols_v * c))


def _ref_layers(net):
    return [(l.w.cpu().numpy().astype(np.float64), l.b.cpu().numpy().astype(np.float64), l.k, l.dil, l.act)
            for l in net.layers]


def test_network_forward_and_gradients_match_reference(sur):
    import torch
    from oracle import surrogate_ref as R
    net = sur.Surrogate(in_ch=2, width=16, out_ch=4, dilations=(1, 2, 5), slope=0.1, seed=3)
    rng = np.random.default_rng(33)
    x = rng.standard_normal((2, 2, 12, 20)).astype(np.float32)
    dy = rng.standard_normal((4, 2, 12, 20)).astype(np.float32)
    y = net.forward(torch.tensor(x, device="cuda"), keep=True)
    dx = net.backward(torch.tensor(dy, device="cuda"), need_dx=True)
    layers = _ref_layers(net)
    ref, trace = R.forward(x, layers, 0.1, bf16=True)
    e = _rel(y.cpu().numpy(), ref)
    _say("forward rel L2 %.2e" % e)
    assert e <= 1e-4
    grads, gx = R.backward(dy, layers, trace, 0.1)
    for l, (gw, gb) in zip(net.layers, grads):
        ew, eb = _rel(l.gw.cpu().numpy(), gw), _rel(l.gb.cpu().numpy(), gb)
        _say("grad rel L2 w %.2e b %.2e" % (ew, eb))
        assert ew <= 1e-2 and eb <= 1e-2
    assert _rel(dx.cpu().numpy(), gx) <= 1e-2


def test_training_learns_a_teacher_network(sur):
    import torch
    teacher = sur.Surrogate(in_ch=2, width=8, out_ch=3, dilations=(1, 2), seed=11)
    student = sur.Surrogate(in_ch=2, width=16, out_ch=3, dilations=(1, 2, 4), seed=12)
    rng = np.random.default_rng(5)
    X = torch.tensor(rng.standard_normal((2, 64, 16, 24)).astype(np.float32), device="cuda")
    T = torch.cat([teacher.forward(X[:, q:q + 16].contiguous()) for q in range(0, 64, 16)], dim=1)
    losses = sur.train(student, X, T, 800, batch=16, lr=3e-3, lr_end=1e-4)
    _say("teacher loss", losses[0], losses[-1])
    assert np.isfinite(losses[-1][1]) and losses[-1][1] < 0.1 * losses[0][1]


def test_surrogate_gain_at_equal_efficiency(sur):
    """What the trained network gains: on the 128 x 128 x 96 surrogate zone,
    surrogate-assisted design (the network trained once on FDTD samples; FDTD
    re-check and gradient every 10 iterations) and plain FDTD-adjoint design,
    both from the same start and each at learning rates 0.02, 0.05, 0.1, to
    the focusing efficiency that 24 plain iterations at 0.02 reach (within
    1 %): at every learning rate the assisted path needs fewer FDTD-adjoint
    evaluations, and its best run fewer than the best plain run."""
    from paper_2501_07979_amd.workloads import c5_zone
    res = sur.equal_efficiency_comparison(c5_zone(), log=lambda m: _say(m))
    p, a, n = res["plain"], res["assisted"], res["surrogate"]
    for pr, ar in zip(p["to_target"], a["to_target"]):
        _say("lr %.3f: plain %d evaluations / %.2f s; assisted %d re-checks + %d surrogate iterations / %.2f s"
             % (pr["lr"], pr["fdtd_evaluations_to_target"], pr["s_to_target"], ar["fdtd_rechecks"],
                ar["surrogate_iterations"], ar["s"]))
    _say("best against best: online speedup %s, with the one-off training %s"
         % (res["speedup_online_best"], res["speedup_with_training_best"]))
    assert p["efficiency_end"] > 10 * p["efficiency_start"]
    assert np.isfinite(n["field_err_median"]) and n["params"] > 1_500_000
    for pr, ar in zip(p["to_target"], a["to_target"]):
        assert pr["lr"] == ar["lr"] and pr["reached"] and ar["reached_target_within_1pct"]
        assert ar["fdtd_rechecks"] < pr["fdtd_evaluations_to_target"]
    assert a["best"]["fdtd_rechecks"] < p["best"]["fdtd_evaluations_to_target"]
