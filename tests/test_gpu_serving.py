"""GPU tests of batched CG and the continuous-batching request loop.

A solve run inside a batch, next to other solves of other sizes, precisions
and stages, must give bitwise the same result as the same solve run alone
(each solve's reductions use only its own work-groups in a fixed order).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


def _alone(fg, micro, N, precision, rtol):
    plan = fg.Plan(len(N), N, precision)
    try:
        return plan.run(micro, rtol=rtol)
    finally:
        plan.close()


def test_batch_alone_equals_mix(fg):
    cases = [(synth.random_circles(1), (41, 41), "fp32"), (synth.random_circles(2), (63, 63), "fp32"),
             (synth.random_circles(3), (21, 21), "fp64"), (synth.random_circles(4), (41, 41), "fp64"),
             (synth.cube_inclusion_aniso(0.5, 3), (9, 9, 9), "fp32"),
             (synth.grf_voxels(7, (45, 45, 45), d=3, corr_len=0.1), (23, 23, 23), "fp32")]
    rtol = 1e-7
    alone = [_alone(fg, m, N, p, rtol) for m, N, p in cases]
    print("alone done", flush=True)
    batch = fg.Batch(capacity=16)
    plans, seqs, k = [], [], []
    for m, N, p in cases:
        pl = fg.Plan(len(N), N, p, stream=batch.stream, P=m.get("P"))
        pl.set_material(m)
        plans.append(pl)
        d = len(N)
        seqs.append([(0, a) for a in range(d)] + [(1, a) for a in range(d)])
        k.append(0)
    owner = {}
    # stagger the starts so that solves of different stages share launches
    for i, pl in enumerate(plans):
        owner[batch.add(pl, *seqs[i][0], rtol=rtol)] = i
        batch.step(3)
        for sid, info, st in batch.poll():
            j = owner.pop(sid)
            k[j] += 1
            if k[j] < len(seqs[j]):
                owner[batch.add(plans[j], *seqs[j][k[j]], rtol=rtol)] = j
    while owner:
        batch.step(5)
        for sid, info, st in batch.poll():
            j = owner.pop(sid)
            k[j] += 1
            if k[j] < len(seqs[j]):
                owner[batch.add(plans[j], *seqs[j][k[j]], rtol=rtol)] = j
    for i, pl in enumerate(plans):
        up, lo, gap = pl.bounds()
        assert np.array_equal(up, alone[i]["upper"]), i
        assert np.array_equal(lo, alone[i]["lower"]), i
        pl.close()
    batch.close()


def test_server_mix_matches_fp64(fg):
    from paper_1412_2033_amd import serve
    reqs = synth.serving_requests(11, 12, rate_per_s=1e6, N_choices=(21, 41, 63))
    # FP32 iterations reach a relative residual of ~1e-6 at contrast 1e4; 5e-6
    # keeps every bound within 1e-6 of the FP64 path (energy error is
    # quadratic in the field error)
    srv = serve.Server(precision="fp32", rtol=5e-6, capacity=8, iters_per_step=6)
    records, stats = srv.run(reqs, realtime=False)
    srv.close()
    assert len(records) == len(reqs)
    assert all(st == 0 for rec in records for st in rec["status"])
    seq, wall = serve.sequential(reqs, precision="fp64", rtol=1e-10)
    by = {r["id"]: r for r in seq}
    worst = 0.0
    for rec in records:
        ref = by[rec["id"]]
        for key in ("upper", "lower"):
            err = np.linalg.norm(rec[key] - ref[key]) / np.linalg.norm(ref[key])
            worst = max(worst, err)
        assert np.min(np.linalg.eigvalsh(rec["upper"] - rec["lower"])) > -1e-12
    print("worst FP32-served vs FP64 bound error %.2e" % worst)
    assert worst < 1e-6


def test_server_3d_mix_under_hbm_budget(fg):
    # 3D random-field requests of three orders arriving at once, with an HBM
    # budget that holds one plan of each order: the second N = 23 request must
    # wait for memory; every result matches the plain FP64 path within 1e-6
    from paper_1412_2033_amd import serve
    reqs = [dict(r, arrival_s=0.0) for r in synth.serving_requests_3d(4, 10, rate_per_s=1.0, N_choices=(5, 13, 23))]
    # the server's plans: small grids concurrent, specialised grids (N = 23: 81^3)
    flags = fg.PRECISIONS["fp32"] | fg.CONCURRENT | fg.FAST_GRID
    need = {N: fg.fftgal_workspace_bytes(3, (N,) * 3, flags) for N in (5, 13, 23)}
    budget = sum(need.values()) + need[5] // 2
    # capacity for all 6 solves of four requests: memory, not slots, defers one
    srv = serve.Server(precision="fp32", rtol=5e-6, capacity=24, iters_per_step=6, hbm_budget=budget)
    records, stats = srv.run(reqs, realtime=False)
    srv.close()
    assert len(records) == len(reqs)
    assert all(st == 0 for rec in records for st in rec["status"])
    assert stats["peak_hbm_bytes"] <= budget
    assert stats["deferred_requests"] >= 1
    seq, _ = serve.sequential(reqs, precision="fp64", rtol=1e-10)
    by = {r["id"]: r for r in seq}
    for rec in records:
        ref = by[rec["id"]]
        for key in ("upper", "lower"):
            assert np.linalg.norm(rec[key] - ref[key]) / np.linalg.norm(ref[key]) < 1e-6
        assert np.min(np.linalg.eigvalsh(rec["upper"] - rec["lower"])) > -1e-12
    with pytest.raises(ValueError):
        small = serve.Server(precision="fp32", hbm_budget=need[5] // 2)
        try:
            small.run(reqs[:1], realtime=False)
        finally:
            small.close()


def _golden_serve_mix():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "serve_mix.json")
    with open(path) as f:
        gold = json.load(f)
    reqs = synth.serving_requests(gold["requests"], gold["n"], rate_per_s=1e6, N_choices=tuple(gold["N_choices"]))
    return reqs, {r["id"]: r for r in gold["results"]}


@pytest.mark.parametrize("precision, rtol, tol", [("fp64", 1e-10, 1e-10), ("fp32", 5e-6, 1e-6)])
def test_served_requests_match_oracle(fg, precision, rtol, tol):
    # eight random-disc requests (N in {21, 41, 123}: double grids 41^2, 81^2
    # and 245^2; contrast 10..1e4) served together in one batch; every entry of
    # every served bound against the oracle's bounds (golden file written by
    # tests/golden/make_golden.py serve_mix, which calls only the oracle)
    from paper_1412_2033_amd import serve
    reqs, gold = _golden_serve_mix()
    srv = serve.Server(precision=precision, rtol=rtol, capacity=8, iters_per_step=6)
    records, stats = srv.run(reqs, realtime=False)
    srv.close()
    assert len(records) == len(reqs)
    worst = 0.0
    for rec in records:
        ref = gold[rec["id"]]
        assert all(st == 0 for st in rec["status"]), rec["status"]
        for key in ("upper", "lower"):
            b = np.asarray(ref[key])
            err = np.max(np.abs(np.asarray(rec[key]) - b)) / np.linalg.norm(b)
            worst = max(worst, err)
            assert err < tol, (rec["id"], rec["N"], key, err)
        assert np.min(np.linalg.eigvalsh(rec["upper"] - rec["lower"])) > -1e-12
    print("%s served vs oracle: worst entry error %.2e" % (precision, worst))


def test_batch_alone_equals_mix_long_lengths(fg):
    # the batched launches at the serving mix's longer double grids (245 and
    # 729, specialised kernels) beside a short one, FP32 and FP64: bitwise the
    # same bounds as each problem solved alone
    cases = [(synth.random_circles(31, contrast=300.0), (123, 123), "fp32"),
             (synth.random_circles(32, contrast=50.0), (365, 365), "fp32"),
             (synth.random_circles(33, contrast=300.0), (123, 123), "fp64"),
             (synth.random_circles(34, contrast=20.0), (41, 41), "fp32")]
    rtol = 5e-6
    alone = [_alone(fg, m, N, p, rtol) for m, N, p in cases]
    print("alone done", flush=True)
    batch = fg.Batch(capacity=16)
    plans = []
    owner = {}
    seqs = []
    k = []
    for i, (m, N, p) in enumerate(cases):
        pl = fg.Plan(len(N), N, p, stream=batch.stream)
        pl.set_material(m)
        plans.append(pl)
        seqs.append([(0, 0), (0, 1), (1, 0), (1, 1)])
        k.append(0)
        owner[batch.add(pl, 0, 0, rtol=rtol)] = i
    while owner:
        batch.step(7)
        for sid, info, st in batch.poll():
            j = owner.pop(sid)
            k[j] += 1
            if k[j] < len(seqs[j]):
                owner[batch.add(plans[j], *seqs[j][k[j]], rtol=rtol)] = j
    for i, pl in enumerate(plans):
        up, lo, gap = pl.bounds()
        assert np.array_equal(up, alone[i]["upper"]), i
        assert np.array_equal(lo, alone[i]["lower"]), i
        pl.close()
    batch.close()
