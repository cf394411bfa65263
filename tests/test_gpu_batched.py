"""Batched uneven products (ozc_zgemm_vbatched / ozc_cgemm_vbatched) through the C-ABI.

Bar: every problem of a batch bit-exact with the CPU oracle (small problems)
and with the single-call path (all sizes); results independent of the
schedule (tile threshold, moduli group, graph or not); graph replays equal to
the eager result with other GPU work in between.
"""
import math
import os

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


@pytest.fixture(scope="module")
def orc():
    from oracle import core

    return core


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nan_a = np.isnan(a.real) | np.isnan(a.imag)
    nan_b = np.isnan(b.real) | np.isnan(b.imag)
    return np.array_equal(nan_a, nan_b) and np.array_equal(a[~nan_a], b[~nan_b])


def _make_batch(seed, count, lo, hi, single=False, ops=True, ab=True, phi_max=4.0):
    """Uneven problems: m, n, k log-uniform in [lo, hi], phi uniform in [0, phi_max]."""
    rng = np.random.default_rng(seed)
    dt = np.complex64 if single else np.complex128
    probs = []
    for p in range(count):
        m, n, k = (int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(3))
        phi = float(rng.uniform(0, phi_max))
        ta = "NTC"[rng.integers(3)] if ops else "N"
        tb = "NTC"[rng.integers(3)] if ops else "N"
        A = workloads.complex_matrix(m, k, phi, seed * 1000 + 3 * p, dtype=dt)
        B = workloads.complex_matrix(k, n, phi, seed * 1000 + 3 * p + 1, dtype=dt)
        C = workloads.complex_matrix(m, n, 1.0, seed * 1000 + 3 * p + 2, dtype=dt)
        alpha = complex(rng.uniform(-2, 2), rng.uniform(-2, 2)) if ab and p % 3 else 1.0
        beta = complex(rng.uniform(-1, 1), rng.uniform(-1, 1)) if ab and p % 2 else 0.0
        probs.append(dict(A=A, B=B, C=C, ta=ta, tb=tb, alpha=alpha, beta=beta))
    return probs


def _upload(probs):
    dev = []
    for q in probs:
        m, k = q["A"].shape
        n = q["B"].shape[1]
        As, Bs = stored(q["A"], q["ta"]), stored(q["B"], q["tb"])
        dA, lda = to_device(As, As.shape[0] + 1)
        dB, ldb = to_device(Bs, Bs.shape[0] + 2)
        dC, ldc = to_device(np.asfortranarray(q["C"]), m + 3)
        dev.append(dict(transa=q["ta"], transb=q["tb"], m=m, n=n, k=k, alpha=q["alpha"],
                        beta=q["beta"], A=dA, lda=lda, B=dB, ldb=ldb, C=dC, ldc=ldc))
    return dev


def _download(dev):
    import torch

    torch.cuda.synchronize()
    return [from_device(d["C"], d["m"], d["n"], d["ldc"]) for d in dev]


def _reset_c(dev, probs):
    for d, q in zip(dev, probs):
        d["C"].copy_(to_device(np.asfortranarray(q["C"]), d["ldc"])[0])


def _single_calls(h, probs, single):
    dev = _upload(probs)
    for d in dev:
        fn = h.cgemm if single else h.zgemm
        fn(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["lda"], d["B"],
           d["ldb"], d["beta"], d["C"], d["ldc"])
    return _download(dev)


@pytest.mark.parametrize("single,mode", [(False, "fast"), (True, "fast"), (False, "accurate"),
                                         (True, "accurate")])
def test_batch_matches_oracle_and_single_calls(handle, orc, single, mode):
    print(f"batched vs oracle single={single} mode={mode}", flush=True)
    N = 8 if single else 14
    handle.set_config(N, mode, "karatsuba")
    handle.set_batch_policy(tile_threshold=160, moduli_group=1, use_graph=True)
    probs = _make_batch(11 + single, 14, 1, 300, single=single)
    probs += _make_batch(15 + single, 2, 170, 260, single=single)
    sizes = [min(q["A"].shape[0], q["B"].shape[1]) for q in probs]
    assert min(sizes) < 160 <= max(sizes)  # both tile sizes (128 and 256) in the batch
    dev = _upload(probs)
    handle.gemm_vbatched(dev, single=single)
    got = _download(dev)
    ref_single = _single_calls(handle, probs, single)
    for p, q in enumerate(probs):
        ref = orc.emulate(q["A"], q["B"], N, mode, alpha=q["alpha"], beta=q["beta"], C=q["C"],
                          single=single)["out"]
        assert _same(got[p], ref), p
        assert _same(got[p], ref_single[p]), p
    info = handle.last_info()
    assert info["num_moduli"] == N and info["int8_ops"] > 0
    handle.set_config(14, "fast", "karatsuba")


def test_schedule_invariance(handle):
    """Tile threshold, moduli group and graph use do not change a single bit."""
    handle.set_config(13, "fast", "karatsuba")
    probs = _make_batch(21, 10, 100, 700)
    dev = _upload(probs)
    results = []
    for thr, grp, graph in [(1 << 30, 1, True), (128, 1, True), (256, 3, False), (512, 13, True)]:
        print(f"schedule thr={thr} group={grp} graph={graph}", flush=True)
        handle.set_batch_policy(tile_threshold=thr, moduli_group=grp, use_graph=graph)
        _reset_c(dev, probs)
        handle.gemm_vbatched(dev)
        results.append(_download(dev))
    for r in results[1:]:
        assert all(_same(a, b) for a, b in zip(results[0], r))


@pytest.mark.parametrize("i", range(int(os.environ.get("OZC_RANDOM_BATCHES", "24"))))
def test_randomized_batches(handle, orc, i):
    """Seeded random batches (1..20 problems of 1..320, both precisions and modes, both
    product forms, tile thresholds that put problems on either tile size, moduli groups,
    graph or not) bit-exact with the oracle problem by problem (24 batches; the
    environment variable OZC_RANDOM_BATCHES runs more)."""
    rng = np.random.default_rng(9100 + i)
    single = bool(rng.random() < 0.4)
    mode = str(rng.choice(["fast", "accurate"]))
    algo = str(rng.choice(["karatsuba", "4m"]))
    N = int(rng.integers(6, 13)) if single else int(rng.integers(10, 21))
    thr = int(rng.choice([64, 128, 160, 256, 1024]))
    grp = int(rng.choice([1, 2, 3, N]))
    graph = bool(rng.random() < 0.5)
    count = int(rng.integers(1, 21))
    print(f"random batch {i}: single={single} mode={mode} algo={algo} N={N} thr={thr} "
          f"group={grp} graph={graph} count={count}", flush=True)
    handle.set_config(N, mode, algo)
    handle.set_batch_policy(tile_threshold=thr, moduli_group=grp, use_graph=graph)
    probs = _make_batch(9200 + i, count, 1, 320, single=single)
    dev = _upload(probs)
    handle.gemm_vbatched(dev, single=single)
    got = _download(dev)
    for p, q in enumerate(probs):
        ref = orc.emulate(q["A"], q["B"], N, mode, algo=algo, alpha=q["alpha"], beta=q["beta"],
                          C=q["C"], single=single)["out"]
        assert _same(got[p], ref), p
    handle.set_batch_policy(tile_threshold=1024, moduli_group=1, use_graph=True)
    handle.set_config(14, "fast", "karatsuba")


def test_expanded_algorithm_batch(handle, orc):
    handle.set_config(10, "fast", "4m")
    handle.set_batch_policy(tile_threshold=1024, moduli_group=2, use_graph=True)
    probs = _make_batch(31, 6, 2, 150)
    dev = _upload(probs)
    handle.gemm_vbatched(dev)
    got = _download(dev)
    for p, q in enumerate(probs):
        ref = orc.emulate(q["A"], q["B"], 10, algo="4m", alpha=q["alpha"], beta=q["beta"],
                          C=q["C"])["out"]
        assert _same(got[p], ref), p
    handle.set_config(14, "fast", "karatsuba")


def test_graph_replays_with_work_in_between(handle):
    """The recorded graph is replayed for an identical call; each replay equals the
    eager result, with unrelated kernels and a single call run between replays."""
    import torch

    handle.set_config(14, "fast", "karatsuba")
    probs = _make_batch(41, 8, 50, 400, ab=False)
    dev = _upload(probs)
    handle.set_batch_policy(tile_threshold=1024, moduli_group=1, use_graph=False)
    handle.gemm_vbatched(dev)
    eager = _download(dev)
    handle.set_batch_policy(tile_threshold=1024, moduli_group=1, use_graph=True)
    other = _make_batch(42, 1, 200, 200, ab=False)[0]
    od = _upload([other])[0]
    for rep in range(4):
        print(f"graph replay {rep}", flush=True)
        for d in dev:
            d["C"].fill_(complex(float("nan"), 0.0))
        handle.gemm_vbatched(dev)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        handle.zgemm("N", "N", od["m"], od["n"], od["k"], 1.0, od["A"], od["lda"], od["B"],
                     od["ldb"], 0.0, od["C"], od["ldc"])
        got = _download(dev)
        assert all(_same(a, b) for a, b in zip(eager, got)), rep


def test_degenerate_problems(handle):
    import torch

    handle.set_config(12, "fast", "karatsuba")
    handle.set_batch_policy(1024, 1, True)
    base = _make_batch(51, 3, 20, 60, ops=False, ab=False)
    probs = [
        dict(base[0]),                                     # ordinary
        dict(base[1], beta=0.5 - 1j, alpha=0.0),          # alpha = 0: C = beta C
        dict(base[2], beta=2.0),                          # ordinary with beta
    ]
    dev = _upload(probs)
    # k = 0 problem and an empty (m = 0) problem
    C0 = workloads.complex_matrix(7, 5, 1.0, 77)
    dC0, ldc0 = to_device(np.asfortranarray(C0), 9)
    dummy = torch.zeros(16, dtype=torch.complex128, device="cuda")
    dev.append(dict(transa="N", transb="N", m=7, n=5, k=0, alpha=1.5, beta=-2.0, A=dummy, lda=7,
                    B=dummy, ldb=1, C=dC0, ldc=ldc0))
    dev.append(dict(transa="N", transb="N", m=0, n=5, k=4, alpha=1.0, beta=0.0, A=dummy, lda=1,
                    B=dummy, ldb=4, C=dummy, ldc=1))
    handle.gemm_vbatched(dev)
    got = _download(dev[:4])
    single = _single_calls(handle, probs, False)
    assert _same(got[0], single[0]) and _same(got[2], single[2])
    assert _same(got[1], single[1])
    exp_k0 = np.array([[complex(np.float64(-2.0) * c.real, np.float64(-2.0) * c.imag)
                        for c in row] for row in C0])
    assert _same(got[3], exp_k0)


def test_argument_errors(handle):
    import paper_2512_08321_amd as ozc

    handle.set_config(14, "fast", "karatsuba")
    probs = _make_batch(61, 2, 10, 20, ops=False)
    dev = _upload(probs)
    bad = [dict(d) for d in dev]
    bad[1]["lda"] = 1  # below the rows of A
    with pytest.raises(ozc.OzcError) as e:
        handle.gemm_vbatched(bad)
    assert e.value.status == 1
    handle.gemm_vbatched([])  # empty batch is a no-op


def test_tuner_policy_keeps_results(handle):
    handle.set_config(14, "fast", "karatsuba")
    handle.set_batch_policy(1024, 1, True)
    probs = _make_batch(71, 12, 64, 1024)
    dev = _upload(probs)
    handle.gemm_vbatched(dev)
    before = _download(dev)
    print("tuning", flush=True)
    pol = handle.batch_tune(dev)
    assert pol["moduli_group"] >= 1 and pol["tile_threshold"] >= 256
    assert handle.batch_policy() == pol
    _reset_c(dev, probs)
    handle.gemm_vbatched(dev)
    after = _download(dev)
    assert all(_same(a, b) for a, b in zip(before, after))


def test_uneven_batch_full_sizes_against_single_calls(handle):
    """The 512-problem workload (m, n, k log-uniform in [64, 2048], phi in [0, 4]):
    every problem bit-identical to its single call."""
    import torch

    handle.set_config(14, "fast", "karatsuba")
    handle.set_batch_policy(1024, 1, True)
    rng = np.random.default_rng(4000)
    dev = []
    for p in range(512):
        m, n, k = (int(round(math.exp(rng.uniform(math.log(64), math.log(2048))))) for _ in range(3))
        phi = float(rng.uniform(0, 4))
        A = workloads.complex_matrix_torch(m, k, phi, 4000 * 1000 + 2 * p)   # column-major m x k
        B = workloads.complex_matrix_torch(k, n, phi, 4000 * 1000 + 2 * p + 1)
        C = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
        dev.append(dict(transa="N", transb="N", m=m, n=n, k=k, alpha=1.0, beta=0.0, A=A, lda=m,
                        B=B, ldb=k, C=C, ldc=m))
    print("batched 512", flush=True)
    handle.gemm_vbatched(dev)
    torch.cuda.synchronize()
    got = [d["C"].clone() for d in dev]
    print("single calls 512", flush=True)
    for d in dev:
        d["C"].zero_()
        handle.zgemm("N", "N", d["m"], d["n"], d["k"], 1.0, d["A"], d["lda"], d["B"], d["ldb"],
                     0.0, d["C"], d["ldc"])
    torch.cuda.synchronize()
    for p, d in enumerate(dev):
        assert torch.equal(torch.view_as_real(got[p]), torch.view_as_real(d["C"])), p


def _log2k_predictor():
    """Parameters of a network whose class is round(log2 k), so that problems with different
    k get different moduli counts (N = 6 + class)."""
    from oracle import mlp

    W1, W2, W3 = (np.zeros((mlp.H, mlp.F)), np.zeros((mlp.H, mlp.H)), np.zeros((mlp.C, mlp.H)))
    W1[0, 2] = 1.0  # feature 2 is log2 k
    W2[0, 0] = 1.0
    c = np.arange(mlp.C, dtype=np.float64)
    W3[:, 0] = 2.0 * c  # z_c = 2 c t - c^2 peaks at c = round(t)
    p = np.concatenate([W1.ravel(), np.zeros(mlp.H), W2.ravel(), np.zeros(mlp.H), W3.ravel(),
                        -c * c, np.zeros(mlp.F), np.ones(mlp.F)]).astype(np.float32)
    assert p.size == mlp.n_params()
    return p


def test_learned_moduli_batch_grouped_expanded(handle):
    """Per-problem moduli counts with moduli groups of 4 and the expanded products: each
    problem bit-identical to a single call at its own count."""
    import paper_2512_08321_amd as ozc

    h2 = ozc.Handle(0)
    try:
        h2.mlp_set_params(_log2k_predictor())
        h2.set_batch_policy(256, 4, True)
        probs = _make_batch(83, 10, 8, 700, phi_max=3.0)
        dev = _upload(probs)
        Ns = [h2.predict_moduli(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["A"],
                                d["lda"], d["B"], d["ldb"]) for d in dev]
        print(f"predicted N {Ns}", flush=True)
        assert len(set(Ns)) >= 3
        h2.set_config(0, "fast", "4m")
        h2.gemm_vbatched(dev)
        got = _download(dev)
        ref_dev = _upload(probs)
        for d, N in zip(ref_dev, Ns):
            h2.set_config(N, "fast", "4m")
            h2.zgemm(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["lda"],
                     d["B"], d["ldb"], d["beta"], d["C"], d["ldc"])
        ref = _download(ref_dev)
        assert all(_same(a, b) for a, b in zip(got, ref))
    finally:
        h2.close()


def test_learned_moduli_batch_matches_single_calls(handle):
    """N = 0 in a batch: each problem runs with its own predicted N, bit-identical to a
    single call at that N."""
    import torch

    import paper_2512_08321_amd as ozc
    from oracle import mlp

    h2 = ozc.Handle(0)
    try:
        h2.mlp_set_params(_log2k_predictor())
        h2.set_batch_policy(1024, 1, True)
        probs = _make_batch(81, 12, 16, 300, phi_max=6.0)
        dev = _upload(probs)
        Ns = [h2.predict_moduli(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["A"],
                                d["lda"], d["B"], d["ldb"]) for d in dev]
        print(f"predicted N {Ns}", flush=True)
        assert len(set(Ns)) >= 2  # one launch sequence serves several moduli counts
        h2.set_config(0, "fast", "karatsuba")
        h2.gemm_vbatched(dev)
        assert h2.last_info()["num_moduli"] == max(Ns)
        got = _download(dev)
        ref_dev = _upload(probs)
        for d, N in zip(ref_dev, Ns):
            h2.set_config(N, "fast", "karatsuba")
            h2.zgemm(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["lda"],
                     d["B"], d["ldb"], d["beta"], d["C"], d["ldc"])
        ref = _download(ref_dev)
        assert all(_same(a, b) for a, b in zip(got, ref))
        torch.cuda.synchronize()
    finally:
        h2.close()


def test_verified_batch_escalates_like_single_calls(handle):
    """Freivalds check in a batch: starting from too few moduli, every problem is rerun with
    two more until its check passes, exactly as a verified single call does (same checks,
    same seed), so each result equals the verified single call's bit for bit."""
    import paper_2512_08321_amd as ozc

    h2 = ozc.Handle(0)
    try:
        probs = _make_batch(91, 8, 16, 200, phi_max=2.0)
        h2.set_config(6, "fast", "karatsuba")
        h2.set_verify(True, 0.0, True)
        dev = _upload(probs)
        h2.gemm_vbatched(dev)
        info = h2.last_info()
        got = _download(dev)
        assert info["verified"] == 1 and info["escalations"] >= 1
        assert info["verify_failed_rows"] == 0 and info["verify_ratio"] <= 1.0
        ref_dev = _upload(probs)
        for d in ref_dev:
            h2.zgemm(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["lda"],
                     d["B"], d["ldb"], d["beta"], d["C"], d["ldc"])
        ref = _download(ref_dev)
        assert all(_same(a, b) for a, b in zip(got, ref))
        # without escalation the same batch ends in VERIFY_FAILED
        h2.set_verify(True, 0.0, False)
        with pytest.raises(ozc.OzcError) as e:
            h2.gemm_vbatched(_upload(probs))
        assert e.value.status == 7
        # a clean batch at 14 moduli passes without reruns and matches the unverified batch
        h2.set_config(14, "fast", "karatsuba")
        h2.set_verify(True, 0.0, True)
        d1 = _upload(probs)
        h2.gemm_vbatched(d1)
        assert h2.last_info()["escalations"] == 0
        h2.set_verify(False)
        d2 = _upload(probs)
        h2.gemm_vbatched(d2)
        assert all(_same(a, b) for a, b in zip(_download(d1), _download(d2)))
    finally:
        h2.close()


@pytest.mark.gpu
@pytest.mark.parametrize("single,mode", [(False, "fast"), (True, "fast"), (False, "accurate")])
def test_verified_batch_check_matches_single_checks(handle, single, mode):
    """The checks of a batch run as one set of launches over all problems, summing each
    product in the same order as a single call's check: the batch's largest residual
    ratio equals the largest over the verified single calls bit for bit, and so do the
    results (all op() forms, alpha/beta, column counts above and below the chunking
    thresholds)."""
    import paper_2512_08321_amd as ozc

    h2 = ozc.Handle(0)
    try:
        print(f"verified batch single={single} mode={mode}", flush=True)
        probs = _make_batch(93 + single, 12, 16, 1500, single=single, phi_max=2.0)
        h2.set_config(9 if single else 14, mode, "karatsuba")
        h2.set_verify(True, 0.0, True)
        dev = _upload(probs)
        h2.gemm_vbatched(dev, single=single)
        info = h2.last_info()
        got = _download(dev)
        ratios, failed = [], 0
        ref_dev = _upload(probs)
        fn = h2.cgemm if single else h2.zgemm
        for d in ref_dev:
            fn(d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["lda"], d["B"],
               d["ldb"], d["beta"], d["C"], d["ldc"])
            si = h2.last_info()
            ratios.append(si["verify_ratio"])
            failed += si["verify_failed_rows"]
        ref = _download(ref_dev)
        assert info["verified"] == 1
        assert info["verify_ratio"] == max(ratios) and 0.0 < info["verify_ratio"] <= 1.0
        assert info["verify_failed_rows"] == failed == 0
        assert all(_same(a, b) for a, b in zip(got, ref))
    finally:
        h2.close()
