"""Continuous-batching server: results are the same alone and in the mix."""
import numpy as np
import pytest
import torch

import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _alone(scene, seq, precision):
    from paper_2312_02999_amd import Solver
    S = Solver(scene, iters=scene.iters, precision=precision)
    R = torch.from_numpy(np.ascontiguousarray(scene.act_R.reshape(-1, 9))).cuda()
    x = torch.from_numpy(np.ascontiguousarray(scene.X)).cuda()
    out = []
    for k, a in enumerate(seq):
        S.set_actuation_scalar(torch.from_numpy(np.ascontiguousarray(a)).cuda(), R if k == 0 else None)
        x = S.solve_frame(x)
        out.append(x.cpu().numpy())
    S.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_results_same_alone_and_in_the_mix(precision):
    from paper_2312_02999_amd.serve import Server, latency_report
    scenes = {"tiny": mg.scene_by_name("tiny"), "slab": mg.slabs(1, nx=6, ny=6, nz=2, iters=12),
              "face": mg.face_like(16, 16, 3, seed=2, slits=(("mouth", 0.0, -0.35, 0.05),), iters=10)}
    reqs = []
    rng = np.random.default_rng(0)
    for k in range(9):
        name = ["tiny", "slab", "face"][k % 3]
        sc = scenes[name]
        scale = 0.5 + 0.5 * rng.random()
        seq = [scale * sc.actuation_at((t + 1) / 3) for t in range(3)]
        reqs.append((name, sc, seq))
    srv = Server(budget_bytes=8 << 30, slots=3, precision=precision)
    futs = [srv.submit(nm, sc, seq) for nm, sc, seq in reqs]
    mixed = [f.result(timeout=300) for f in futs]
    rep = latency_report(srv.completed)
    srv.close()
    assert rep["requests"] == 9 and rep["frames"] == 27
    for (nm, sc, seq), got in zip(reqs, mixed):
        ref = _alone(sc, seq, precision)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), nm


def test_admission_rejects_oversized_request_and_evicts():
    from paper_2312_02999_amd.serve import Server, estimate_bytes
    tiny = mg.scene_by_name("tiny")
    slab = mg.slabs(1, nx=6, ny=6, nz=2, iters=8)
    budget = max(estimate_bytes(tiny), estimate_bytes(slab)) + (1 << 20)
    srv = Server(budget_bytes=budget, slots=1, precision=0)
    f1 = srv.submit("tiny", tiny, [tiny.actuation_at(0.5)])
    f2 = srv.submit("slab", slab, [slab.actuation_at(0.5)])     # needs the tiny solver evicted
    assert len(f1.result(timeout=120)) == 1 and len(f2.result(timeout=120)) == 1
    assert srv.used <= budget
    small = Server(budget_bytes=1 << 20, slots=1, precision=0)
    f3 = small.submit("tiny", tiny, [tiny.actuation_at(0.5)])
    with pytest.raises(MemoryError):
        f3.result(timeout=60)
    srv.close()
    small.close()
