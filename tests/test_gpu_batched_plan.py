"""GPU tests of the batch plan (lstsq_batched_create / bind / launch / results):
the batched sketch-and-solve captured into one HIP graph.

  * a mixed batch (k from 16 to 256, float32 / float64 / bfloat16, n from a
    few thousand rows to a few hundred thousand, ragged last tiles) runs as
    ONE graph launch, and every problem matches the oracle's sketch-and-solve
    on the oracle's own S A and S b for the same sketch (float64 to 1e-11
    relative; float32 / bfloat16 within the first-order perturbation bound of
    the small least-squares problem, as in the other batched tests);
  * block counts zeta = 1, 2, 3, 8 and 16 (one to sixteen waves a workgroup,
    bucket parts, two block groups) against the oracle;
  * launches replay bitwise, also from a graph the caller captures around
    lstsq_batched_enqueue, and agree with the one-call lstsq_sketch_solve_batched;
  * a rank-deficient problem inside the plan takes the SVD fallback and
    matches the oracle's truncated solution;
  * the tuner times the batch's classes, writes its JSON cache, and later
    plans read it back;
  * the launch's device time is reported for every problem.
"""
import json

import numpy as np
import pytest
import torch

from oracle import lstsq as ol
from oracle import sketches as sk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


def _problem(n, k, dtype, seed, dependent=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, k))
    if dependent:
        A[:, k - 1] = 2.0 * A[:, 0]
    b = A @ rng.standard_normal(k) + 1e-4 * rng.standard_normal(n)
    return torch.from_numpy(A).to(dtype).cuda(), torch.from_numpy(b).to(dtype).cuda()


def _oracle(A64, b64, d, zeta, seed, u):
    SA = sk.sparsestack_apply(A64, d, zeta, seed)
    Sb = sk.sparsestack_apply(b64[:, None], d, zeta, seed)[:, 0]
    x, r, s = ol.sketch_and_solve(SA, Sb)
    Sabs = abs(sk.sparsestack_csr(A64.shape[0], d, zeta, seed))
    cnt = np.asarray((Sabs != 0).sum(axis=1)).ravel()[:, None]
    E = np.linalg.norm((cnt + 8.0) * u * (Sabs @ np.abs(A64)))
    e = np.linalg.norm((cnt[:, 0] + 8.0) * u * (Sabs @ np.abs(b64)))
    res = np.linalg.norm(SA @ x - Sb)
    smin = s[r - 1]
    tol = 2.0 * ((E * np.linalg.norm(x) + e) / smin + E * res / smin ** 2)
    return x, r, tol


def _check(problems, xs, ranks, d_per_k, zeta, shapes):
    for (A, b, seed), x, rank, (n, k, dt) in zip(problems, xs, ranks, shapes):
        A64 = A.to(torch.float64).cpu().numpy()
        b64 = b.to(torch.float64).cpu().numpy()
        xg = x.cpu().numpy()
        if dt == torch.float64:
            xr, r, _ = _oracle(A64, b64, d_per_k * k, zeta, seed, 2.0 ** -53)
            assert np.linalg.norm(xg - xr) <= 1e-11 * np.linalg.norm(xr), (n, k, dt)
        else:
            xr, r, tol = _oracle(A64, b64, d_per_k * k, zeta, seed, 2.0 ** -24)
            assert np.linalg.norm(xg - xr) <= tol, (n, k, dt)
        assert rank == r == k


MIXED = [(250001, 256, torch.float32), (70003, 230, torch.float32), (5000, 16, torch.float32),
         (120000, 200, torch.float32), (33333, 191, torch.float32), (9001, 64, torch.float32),
         (41000, 127, torch.float32), (16384, 128, torch.float32), (20011, 65, torch.float64),
         (30000, 256, torch.float64), (12000, 150, torch.bfloat16), (7777, 33, torch.float32),
         (100000, 100, torch.bfloat16), (3001, 255, torch.float32)]


@pytest.fixture(scope="module")
def mixed(lib):
    problems = []
    for i, (n, k, dt) in enumerate(MIXED):
        A, b = _problem(n, k, dt, 300 + i)
        problems.append((A, b, 5000 + i))
    plan = lib.BatchPlan(problems, 4, 4, lib.SK_BATCH_NOTUNE)
    plan.bind()
    plan.launch()
    status, ranks, t_ms, rc = plan.results()
    return problems, plan, status, ranks, t_ms, rc


def test_plan_one_graph_launch_matches_oracle(lib, mixed):
    problems, plan, status, ranks, t_ms, rc = mixed
    assert rc == 0 and status == [0] * len(MIXED)
    inf = plan.info()
    assert inf.graph_launches == 1 and inf.kernel_nodes >= 8
    assert inf.sketch_workgroups >= 1 and inf.solve_workgroups == len(MIXED) and inf.reduce_items > 0
    _check(problems, plan.xs, ranks, 4, 4, MIXED)
    assert all(t > 0.0 for t in t_ms)


def test_plan_replays_bitwise_and_matches_one_call(lib, mixed, tmp_path, monkeypatch):
    monkeypatch.setenv("SKETCH_TUNE_CACHE", str(tmp_path / "none.json"))  # the one call: default tiles
    problems, plan, status, ranks, t_ms, rc = mixed
    first = [x.clone() for x in plan.xs]
    for rep in range(3):
        for x in plan.xs:
            x.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")  # eager work between the launches
        (junk * 2).sum().item()
        plan.launch()
        st, rk, _, rc2 = plan.results()
        assert rc2 == 0 and rk == ranks
        for a, b in zip(first, plan.xs):
            assert torch.equal(a, b)
    assert plan.info().graph_launches == 4
    xs1 = lib.solve_batched(problems)[0]
    for a, b in zip(first, xs1):
        assert torch.equal(a, b)


def test_plan_enqueue_captured_by_the_caller(lib, mixed):
    problems, plan, status, ranks, t_ms, rc = mixed
    first = [x.clone() for x in plan.xs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.enqueue(torch.cuda.current_stream())
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for x in plan.xs:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(first, plan.xs):
            assert torch.equal(a, b)
    st, rk, _, rc2 = plan.results()
    assert rc2 == 0 and rk == ranks


WAVE_SHAPES = [  # zeta, d_per_k, two problems each (d_per_k * k divisible by zeta)
    (1, 8, [(9000, 24, torch.float32), (4517, 27, torch.float32)]),     # 1 wave a unit; 2 parts
    (2, 4, [(11000, 40, torch.float32), (5517, 43, torch.float32)]),    # 2 waves a unit
    (3, 6, [(6000, 30, torch.float64), (3017, 33, torch.float64)]),     # 4 waves, one idle
    (8, 4, [(15000, 70, torch.float32), (7517, 72, torch.float32)]),    # 8 waves a unit
    (16, 4, [(8000, 36, torch.float32), (4017, 40, torch.float32)]),    # two block groups
    (4, 4, [(4000, 20, torch.bfloat16), (2017, 22, torch.bfloat16)]),
]


@pytest.mark.parametrize("zeta,d_per_k,shapes", WAVE_SHAPES)
def test_plan_wave_shapes_match_oracle(lib, zeta, d_per_k, shapes):
    problems = []
    for i, (n, k, dt) in enumerate(shapes):
        A, b = _problem(n, k, dt, 700 + 10 * zeta + i)
        problems.append((A, b, 9000 + zeta + i))
    plan = lib.BatchPlan(problems, d_per_k, zeta, lib.SK_BATCH_NOTUNE)
    plan.bind()
    plan.launch()
    status, ranks, _, rc = plan.results()
    assert rc == 0 and status == [0, 0]
    _check(problems, plan.xs, ranks, d_per_k, zeta, shapes)


def test_autotune_writes_and_reuses_the_cache(lib, tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SKETCH_TUNE_CACHE", str(path))
    shapes = [(60000, 100, torch.float32), (40000, 220, torch.float32), (30000, 50, torch.float32)]
    problems = []
    for i, (n, k, dt) in enumerate(shapes):
        A, b = _problem(n, k, dt, 900 + i)
        problems.append((A, b, 9900 + i))
    plan = lib.BatchPlan(problems, 4, 4, lib.SK_BATCH_AUTOTUNE)
    assert plan.info().tuned == len(shapes)
    entries = json.loads(path.read_text())
    assert len(entries) == 3  # classes: 128-slot file, 200-slot file in two parts, 64-slot file
    assert {key.split("/", 2)[2] for key in entries} == {"r128/p1", "r200/p2", "r64/p1"}
    for key, v in entries.items():
        assert v["chunk_d"] in (8, 16, 32) and v["ms"] > 0
    plan.bind()
    plan.launch()
    status, ranks, _, rc = plan.results()
    assert rc == 0
    _check(problems, plan.xs, ranks, 4, 4, shapes)
    again = lib.BatchPlan(problems, 4, 4, 0)
    assert again.info().tuned == len(shapes)
    assert lib.BatchPlan(problems, 4, 4, lib.SK_BATCH_NOTUNE).info().tuned == 0


def test_plan_rank_deficient_problem_takes_the_svd(lib):
    """A problem whose last column repeats its first fails the full-rank certificate inside the graph; the SVD
    fallback kernel gives it the oracle's truncated solution and rank k - 1, and its neighbour is unaffected."""
    good = _problem(3000, 12, torch.float64, 11)
    bad = _problem(3000, 12, torch.float64, 12, dependent=True)
    problems = [(*good, 21), (*bad, 22)]
    plan = lib.BatchPlan(problems, 4, 4, lib.SK_BATCH_NOTUNE)
    plan.bind()
    plan.launch()
    status, ranks, _, rc = plan.results()
    assert rc == lib.SK_W_RANKDEF
    assert status == [0, lib.SK_W_RANKDEF] and ranks == [12, 11]
    for (A, b, seed), x, rank in zip(problems, plan.xs, ranks):
        xr, r, _ = _oracle(A.cpu().numpy(), b.cpu().numpy(), 48, 4, seed, 2.0 ** -53)
        assert r == rank and np.linalg.norm(x.cpu().numpy() - xr) <= 1e-9 * np.linalg.norm(xr)


def test_plan_refuses_oversized_sketch_and_small_workspace(lib):
    A, b = _problem(4000, 300, torch.float32, 1)
    with pytest.raises(lib.SketchError):
        lib.BatchPlan([(A, b, 1)], 4, 4)  # d = 1200 > 1024
    A, b = _problem(4000, 30, torch.float32, 2)
    plan = lib.BatchPlan([(A, b, 1)], 4, 4)
    ws = torch.empty(plan.workspace_bytes() // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.SketchError):
        plan.bind(ws)
    with pytest.raises(lib.SketchError):
        plan.launch()
    plan.bind()
    with pytest.raises(lib.SketchError):
        plan.results()  # bound, but nothing launched yet
