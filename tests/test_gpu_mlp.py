"""Moduli-count predictor on the GPU (through the C-ABI) against the CPU FP64 reference.

Bar (FP32 kernels against FP64 references): statistics to 1e-5 relative;
logits, gradients and one Adam step to 1e-4 relative to the largest entry.
The learned choice runs the emulation with the predicted N, bit-exact with
the oracle at that N; labels are certified against the 24-moduli reference
and agree with the oracle's exact emulation and double-double product; a
small end-to-end run shows the trained network using fewer moduli than the
fixed rule with every result accepted by the same check.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import from_device, stored, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import torch

    import paper_2512_08321_amd as ozc

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = ozc.Handle(0)
    yield h
    torch.cuda.synchronize()
    h.close()


def _rand_params(seed):
    from oracle import mlp

    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.n_params()).astype(np.float32)
    n = mlp.n_params()
    p[n - 2 * mlp.F:n - mlp.F] = rng.normal(0, 1, mlp.F)
    p[n - mlp.F:] = rng.uniform(0.5, 2.0, mlp.F)
    return p


@pytest.mark.parametrize("case", ["NN", "TC", "zeros", "single", "skewed"])
def test_features_match_oracle(handle, case):
    import torch

    from oracle import features as ft

    print(f"features {case}", flush=True)
    single = case == "single"
    dt = np.complex64 if single else np.complex128
    A = workloads.complex_matrix(70, 3000, 2.0, 101, dtype=dt)
    B = workloads.complex_matrix(3000, 45, 2.0, 102, dtype=dt)
    ta, tb = ("T", "C") if case == "TC" else ("N", "N")
    if case == "zeros":
        A[3] = 0
        A[:, 5] = 0
        B[:, 7] = 0
    if case == "skewed":
        rng = np.random.default_rng(103)
        A = workloads.skewed(A, col_exp=rng.integers(-40, 1, 3000))
    As, Bs = stored(A, ta), stored(B, tb)
    dA, lda = to_device(As)
    dB, ldb = to_device(Bs)
    out = torch.empty(20, dtype=torch.float32, device="cuda")
    handle.features(ta, tb, 70, 45, 3000, dA, lda, dB, ldb, out, single=single)
    got = out.cpu().numpy().astype(np.float64)
    ref = ft.features(A, B)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5), np.c_[got, ref]


def test_features_reproducible_and_match_oracle_long_k(handle):
    """Row sums accumulated by many blocks (k = 40000: 20 chunks per row of B, 157 per
    row of A) in fixed point: repeated calls give identical bits, and the statistics
    still match the FP64 reference."""
    import torch

    from oracle import features as ft

    A = workloads.complex_matrix(300, 40000, 3.0, 104)
    B = workloads.complex_matrix(40000, 33, 3.0, 105)
    dA, lda = to_device(stored(A, "N"))
    dB, ldb = to_device(stored(B, "N"))
    outs = []
    for _ in range(4):
        out = torch.empty(20, dtype=torch.float32, device="cuda")
        handle.features("N", "N", 300, 33, 40000, dA, lda, dB, ldb, out)
        outs.append(out.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    ref = ft.features(A, B)
    got = outs[0].astype(np.float64)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5), np.c_[got, ref]


def test_forward_and_gradient_match_oracle(handle):
    import torch

    from oracle import mlp

    p = _rand_params(7)
    handle.mlp_set_params(p)
    assert np.array_equal(handle.mlp_get_params(), p)
    rng = np.random.default_rng(8)
    X = rng.normal(0, 2, (37, mlp.F)).astype(np.float32)
    y = rng.integers(0, mlp.C, 37).astype(np.int32)
    dX, dy = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    z = torch.empty((37, mlp.C), dtype=torch.float32, device="cuda")
    handle.mlp_forward(dX, 37, z)
    zr, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.allclose(z.cpu().numpy(), zr, rtol=1e-4, atol=1e-4 * np.abs(zr).max())
    g = torch.empty(mlp.n_params(), dtype=torch.float32, device="cuda")
    loss = handle.mlp_grad(dX, dy, 37, g)
    gr = mlp.grad(p.astype(np.float64), X.astype(np.float64), y)
    assert loss == pytest.approx(mlp.loss(p.astype(np.float64), X.astype(np.float64), y), rel=1e-4)
    assert np.allclose(g.cpu().numpy(), gr, rtol=0, atol=1e-4 * np.abs(gr).max())


def test_one_adam_step_matches_oracle(handle):
    import torch

    from oracle import mlp

    p = _rand_params(9)
    handle.mlp_set_params(p)
    rng = np.random.default_rng(10)
    X = rng.normal(0, 1, (50, mlp.F)).astype(np.float32)
    y = rng.integers(0, mlp.C, 50).astype(np.int32)
    handle.mlp_train(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), 50, epochs=1,
                     batch=64, lr=1e-3, init=False)
    got = handle.mlp_get_params()
    pd = p.astype(np.float64)
    g = mlp.grad(pd, X.astype(np.float64), y)
    n_train = mlp.n_params() - 2 * mlp.F
    want, _, _ = mlp.adam(pd, g, np.zeros_like(pd), np.zeros_like(pd), 1, lr=1e-3, n_train=n_train)
    # the first step moves every trainable entry by about lr sign(g): compare the moves
    assert np.allclose(got - p, want - pd, rtol=0, atol=2e-5)


def test_training_learns_a_separable_rule(handle):
    import torch

    from oracle import mlp

    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (4000, mlp.F)).astype(np.float32)
    W = rng.normal(0, 1, (mlp.C, mlp.F))
    y = np.argmax(X @ W.T, axis=1).astype(np.int32)
    dX, dy = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    losses = handle.mlp_train(dX, dy, 4000, epochs=30, batch=128, lr=3e-3, seed=5)
    assert losses[-1] < 0.5 * losses[0]
    z = torch.empty((4000, mlp.C), dtype=torch.float32, device="cuda")
    handle.mlp_forward(dX, 4000, z)
    acc = float((z.argmax(dim=1).cpu().numpy() == y).mean())
    ref_pred = mlp.predict(handle.mlp_get_params().astype(np.float64), X.astype(np.float64))
    assert acc > 0.8
    assert float((ref_pred == z.argmax(dim=1).cpu().numpy()).mean()) > 0.99


def test_auto_moduli_runs_the_predicted_count(handle):
    """N = 0: the call runs with the predicted N (bit-exact with the oracle at that N);
    without parameters it uses the fallback."""
    import torch

    import paper_2512_08321_amd as ozc
    from oracle import core

    A = workloads.complex_matrix(96, 200, 1.0, 121)
    B = workloads.complex_matrix(200, 64, 1.0, 122)
    dA, lda = to_device(A)
    dB, ldb = to_device(B)
    dC, ldc = to_device(np.zeros((96, 64), complex))
    h2 = ozc.Handle(0)
    try:
        h2.set_auto_moduli(fallback=15, margin=0)
        h2.set_config(0, "fast", "karatsuba")
        h2.zgemm("N", "N", 96, 64, 200, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc)
        torch.cuda.synchronize()
        assert h2.last_info()["num_moduli"] == 15
        p = _rand_params(12)
        h2.mlp_set_params(p)
        N = h2.predict_moduli("N", "N", 96, 64, 200, dA, lda, dB, ldb)
        assert 6 <= N <= 24
        # the fused inference launch picks the class of the layered forward pass
        feat = torch.empty(20, dtype=torch.float32, device="cuda")
        h2.features("N", "N", 96, 64, 200, dA, lda, dB, ldb, feat)
        logits = torch.empty(ozc.MLP_CLASSES, dtype=torch.float32, device="cuda")
        h2.mlp_forward(feat, 1, logits)
        assert N == min(24, ozc.MLP_MIN_N + int(torch.argmax(logits).item()))
        h2.zgemm("N", "N", 96, 64, 200, 1.0, dA, lda, dB, ldb, 0.0, dC, ldc)
        torch.cuda.synchronize()
        assert h2.last_info()["num_moduli"] == N
        got = from_device(dC, 96, 64, ldc)
        assert np.array_equal(got, core.emulate(A, B, N)["out"])
    finally:
        h2.close()


def test_trained_predictor_beats_fixed_rule(handle):
    """Small end-to-end run: label instances with certified labels, train, and run held-out
    instances with the learned N (plus a margin of 1) and the Freivalds check at the target
    (escalation by 2 on failure).  Every call ends accepted by the check, and the exact
    (rational) row test of the oracle accepts the same results; the mean N stays below the
    fixed rule's.  The check aggregates a row, so it cannot see a single entry over the
    per-entry target: every per-entry miss must be an instance whose learned N fell below
    its certified minimum (the miss rate is printed)."""
    import paper_2512_08321_amd as ozc
    from oracle import freivalds
    from paper_2512_08321_amd import autoN

    h2 = ozc.Handle(0)
    try:
        target = 1e-15
        kw = dict(lo=48, hi=192, klo=64, khi=2048, phi_max=8.0, skew_max=40)
        print("labelling training instances", flush=True)
        X, y, meta = autoN.generate(h2, 360, seed=2024, target=target, **kw)
        N_train = [r[-1] for r in meta]
        n_fix = autoN.fixed_rule(N_train)
        h2.mlp_train(X, y, len(meta), epochs=150, batch=64, lr=3e-3, seed=7)
        rng = np.random.default_rng(99)
        insts = [autoN.draw_instance(rng, **kw) for _ in range(40)]
        print("evaluating held-out instances", flush=True)
        res = autoN.evaluate(h2, insts, target, margin=1,
                             check=lambda inst, C: C.cpu().numpy().T.copy())
        used = np.array([r["N_used"] for r in res])
        assert all(r["status"] == 0 for r in res)
        for inst, r in list(zip(insts, res))[:8]:   # the exact row test on a subset
            A = inst["A"].cpu().numpy().T
            B = inst["B"].cpu().numpy().T
            assert freivalds.check(A, B, r["check"], seed=0x5EED, rel=target)[1] == 0
        labels = [autoN.label(h2, inst, target) for inst in insts]
        misses = [i for i, r in enumerate(res) if r["err"] > target]
        print(f"fixed rule N={n_fix}; learned mean N={used.mean():.2f}; escalated "
              f"{sum(r['esc'] > 0 for r in res)}/{len(res)}; per-entry target missed on "
              f"{len(misses)}/{len(res)} (certified bound)", flush=True)
        assert all(res[i]["N_used"] < labels[i] for i in misses)
        assert used.mean() < n_fix
    finally:
        h2.close()


def test_certified_labels_against_the_oracle(handle):
    """The library's labels (certified bound on the 24-moduli reference) against the
    minimal N the oracle finds with the exact emulation and the double-double product:
    never below it (the bound is conservative), at most two above, and the oracle's error
    at the label meets the target."""
    from oracle import core
    from paper_2512_08321_amd import autoN

    target = 1e-15
    rng = np.random.default_rng(31)
    gaps = []
    for t in range(16):
        inst = autoN.draw_instance(rng, lo=16, hi=48, klo=16, khi=400, phi_max=8.0, skew_max=40)
        L = autoN.label(handle, inst, target)
        A = inst["A"].cpu().numpy().T
        B = inst["B"].cpu().numpy().T
        hi, lo = core.dd_gemm(A, B)
        ab = core.abs_product(A, B)
        errs = {N: core.err_nc(core.emulate(A, B, N)["out"], hi, lo, ab) for N in range(6, 25)}
        ok = [N for N in range(6, 25) if errs[N] <= target]
        N_or = ok[0] if ok else 25
        print(f"instance {t}: m={inst['m']} k={inst['k']} phi={inst['phi']:.2f} "
              f"skew={inst['sigma']} label={L} oracle={N_or}", flush=True)
        assert N_or <= L <= N_or + 2
        if L <= 24:
            assert errs[L] <= target
        gaps.append(L - N_or)
    print(f"label - oracle minimum: {np.bincount(gaps).tolist()}", flush=True)


def test_fused_inference_many_rows(handle):
    """ozc_mlp_predict (the fused launch of the per-call prediction) on 4000 feature rows:
    the class of every row equals the argmax of ozc_mlp_forward's logits, and the FP64
    oracle's class wherever the oracle's two best logits are not within FP32 noise."""
    import torch

    from oracle import mlp

    p = _rand_params(17)
    handle.mlp_set_params(p)
    rng = np.random.default_rng(18)
    X = rng.normal(0, 2, (4000, mlp.F)).astype(np.float32)
    dX = torch.from_numpy(X).cuda()
    cls = torch.empty(4000, dtype=torch.int32, device="cuda")
    handle.mlp_predict(dX, 4000, cls)
    z = torch.empty((4000, mlp.C), dtype=torch.float32, device="cuda")
    handle.mlp_forward(dX, 4000, z)
    got = cls.cpu().numpy()
    assert np.array_equal(got, z.argmax(dim=1).cpu().numpy())
    zr, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    top = np.sort(zr, axis=1)
    clear = (top[:, -1] - top[:, -2]) > 1e-4 * np.abs(zr).max()
    ref = np.argmax(zr, axis=1)
    assert np.array_equal(got[clear], ref[clear])
    near = ~clear   # a near tie: the chosen class is one of the tied best
    assert all(zr[i, got[i]] >= top[i, -1] - 1e-4 * np.abs(zr).max() for i in np.flatnonzero(near))
    assert clear.mean() > 0.99


def test_save_and_load_round_trip(handle, tmp_path):
    """A saved network loads bit-identically into a new handle (same logits); files
    that are truncated, corrupted, of other dimensions or with trailing bytes are
    rejected without touching the loaded parameters."""
    import struct

    import torch

    import paper_2512_08321_amd as ozc
    from oracle import mlp

    p = _rand_params(13)
    handle.mlp_set_params(p)
    path = tmp_path / "mlp.bin"
    handle.mlp_save(path)
    raw = path.read_bytes()
    P = mlp.n_params()
    assert len(raw) == 8 + 5 * 4 + 4 * P + 8
    assert raw[:8] == b"OZCMLP01"
    assert struct.unpack("<5i", raw[8:28]) == (mlp.F, mlp.H, mlp.C, ozc.MLP_MIN_N, P)
    assert np.array_equal(np.frombuffer(raw[28:28 + 4 * P], "<f4"), p)

    h2 = ozc.Handle(0)
    try:
        with pytest.raises(ozc.OzcError):
            h2.mlp_save(tmp_path / "none.bin")  # no parameters yet
        h2.mlp_load(path)
        assert np.array_equal(h2.mlp_get_params(), p)
        X = torch.from_numpy(np.random.default_rng(14).normal(0, 1, (9, mlp.F)).astype(np.float32)).cuda()
        z1 = torch.empty((9, mlp.C), dtype=torch.float32, device="cuda")
        z2 = torch.empty_like(z1)
        handle.mlp_forward(X, 9, z1)
        h2.mlp_forward(X, 9, z2)
        assert torch.equal(z1, z2)

        q = _rand_params(15)
        h2.mlp_set_params(q)
        bad = {
            "truncated": raw[:-9],
            "trailing": raw + b"\0",
            "magic": b"X" + raw[1:],
            "dims": raw[:8] + struct.pack("<i", mlp.F + 1) + raw[12:],
            "flipped": raw[:100] + bytes([raw[100] ^ 1]) + raw[101:],
        }
        for name, data in bad.items():
            f = tmp_path / f"{name}.bin"
            f.write_bytes(data)
            with pytest.raises(ozc.OzcError):
                h2.mlp_load(f)
            assert np.array_equal(h2.mlp_get_params(), q), name
        with pytest.raises(ozc.OzcError):
            h2.mlp_load(tmp_path / "missing.bin")
    finally:
        h2.close()
