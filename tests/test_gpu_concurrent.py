"""GPU tests of concurrent solves (plans made with FFTGAL_CONCURRENT).

The d primal and d dual solves of a microstructure are independent (Cor.
Ga_linsys).  A concurrent plan keeps one set of per-solve buffers per solve,
so fftgal_solve_all runs all 2d solves in shared launches and a batch can
hold all of them at once.  Each solve keeps its own reductions, so every
result must equal bitwise the result of the solves run one after another, in
FP64 and in the FP32-iteration form (whose best-iterate checkpoints run at
the same iteration counts).
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


CASES = [
    ("disc2d_N41_fp64", lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (41, 41), "fp64", 1e-10),
    ("disc2d_N1013_fp64", lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (1013, 1013), "fp64", 1e-10),
    ("circles2d_N63_fp32", lambda: synth.random_circles(5), (63, 63), "fp32", 1e-7),
    ("aniso3d_N23_fp32", lambda: synth.cube_inclusion_aniso(0.45, 4), (23, 23, 23), "fp32", 5e-6),
    ("vox3d_N21_fp64", lambda: synth.grf_voxels(6, (41, 41, 41), d=3, corr_len=0.1), (21, 21, 21), "fp64", 1e-9),
    # the 225-point tiles of both strided passes (7 FP64 / 9 FP32 pencils,
    # ragged at these pencil counts) and the 729-point FP32 tiles, several
    # problems per launch
    ("vox3d_N113x113x5_fp64", lambda: synth.grf_voxels(8, (225, 225, 9), d=3, corr_len=0.1), (113, 113, 5),
     "fp64", 1e-9),
    ("vox3d_N113x113x5_fp32", lambda: synth.grf_voxels(8, (225, 225, 9), d=3, corr_len=0.1), (113, 113, 5),
     "fp32", 5e-6),
    ("circles2d_N365_fp32", lambda: synth.random_circles(9, contrast=30.0), (365, 365), "fp32", 5e-6),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_solve_all_equals_one_after_another(fg, k):
    name, make, N, precision, rtol = CASES[k]
    micro = make()
    print("concurrent %s" % name, flush=True)
    res = {}
    for conc in (False, True):
        plan = fg.Plan(len(N), N, precision, P=micro.get("P"), concurrent=conc)
        try:
            res[conc] = plan.run(micro, rtol=rtol)
        finally:
            plan.close()
    a, b = res[False], res[True]
    assert [i["iters"] for i in a["info_primal"] + a["info_dual"]] == \
        [i["iters"] for i in b["info_primal"] + b["info_dual"]]
    assert np.array_equal(a["upper"], b["upper"]) and np.array_equal(a["lower"], b["lower"])


def test_concurrent_server_equals_single_slot_server(fg):
    # the serving loop adding all 2d solves of a request at once gives bitwise
    # the bounds of the loop that chains them
    from paper_1412_2033_amd import serve
    reqs = synth.serving_requests(13, 10, rate_per_s=1e6, N_choices=(21, 41, 63))
    out = {}
    for conc in (False, True):
        srv = serve.Server(precision="fp32", rtol=5e-6, capacity=16, iters_per_step=5, concurrent=conc)
        records, stats = srv.run(reqs, realtime=False)
        srv.close()
        out[conc] = {r["id"]: r for r in records}
    for rid, r in out[True].items():
        assert np.array_equal(r["upper"], out[False][rid]["upper"]), rid
        assert np.array_equal(r["lower"], out[False][rid]["lower"]), rid


def test_solve_slot_errors(fg):
    micro = synth.square_inclusion(2, 0.6, 1.0, 10.0)
    single = fg.Plan(2, (9, 9), "fp64")
    conc = fg.Plan(2, (9, 9), "fp64", concurrent=True, stream=single.stream)
    batch = fg.Batch(capacity=8, stream=single.stream)
    try:
        single.set_material(micro)
        conc.set_material(micro)
        batch.add(single, 0, 0)
        with pytest.raises(fg.FftgalError) as e:
            batch.add(single, 0, 1)  # one solve slot
        assert e.value.code == -5
        for kind in (0, 1):
            for a in (0, 1):
                batch.add(conc, kind, a)
        with pytest.raises(fg.FftgalError) as e:
            batch.add(conc, 1, 1)  # already in the batch
        assert e.value.code == -5
        with pytest.raises(fg.FftgalError) as e:
            conc.solve_primal(0)  # the plan's solves are in a batch
        assert e.value.code == -5
        while batch.step(10) > 0:
            pass
        assert len(batch.poll()) == 5
        conc.bounds()
    finally:
        batch.close()
        single.close()
        conc.close()
    with pytest.raises(fg.FftgalError):
        fg.Plan(2, (9, 9), "fp64", scheme="reduced", concurrent=True)
