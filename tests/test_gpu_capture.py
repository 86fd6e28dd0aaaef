"""Stream capture of the sketch and of sketch-and-solve (Alg. 3) into one HIP
graph, through the C-ABI, with caller workspaces: sketch_apply (ws given) and
lstsq_sketch_solve_async enqueue everything on the capturing stream with no
allocation and no host synchronization. The graph is replayed three times,
with the program's own eager work (overwriting the outputs) and a
synchronization between replays; every replay gives bitwise the eager
results, which in turn equal lstsq_sketch_solve's x and rank. Also: the async
solve refuses a missing or too small workspace before enqueuing anything."""
import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lib():
    from paper_2508_21189_amd import libsketch
    libsketch.load()
    return libsketch


@pytest.mark.parametrize("n,m,d,zeta,seed", [(200003, 64, 256, 8, 1), (70001, 30, 120, 4, 2)])
def test_apply_and_solve_under_capture(lib, n, m, d, zeta, seed):
    from paper_2508_21189_amd import inputs
    A_h, b_h, _ = inputs.small_gaussian(n, m, seed=seed)
    A = torch.from_numpy(A_h).cuda()
    b = torch.from_numpy(b_h).cuda()
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    ws_a = torch.empty(S.workspace_size(0, torch.float64, m), dtype=torch.uint8, device="cuda")
    ws_s = torch.empty(S.solve_workspace_size(m), dtype=torch.uint8, device="cuda")
    # eager references
    SA_e = S.apply(A, ws=ws_a)
    x_e = torch.empty(m, dtype=torch.float64, device="cuda")
    res_e = torch.zeros(lib.SOLVE_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    S.lstsq_solve_async(A, b, x_e, ws_s, result=res_e)
    torch.cuda.synchronize()
    x_sync, rc, info = S.lstsq_solve(A, b)
    assert torch.equal(x_e, x_sync)
    r_e, smax_e, smin_e = lib.read_solve_result(res_e)
    assert r_e == info["rank"] == m and smax_e == info["sigma_max"] and smin_e == info["sigma_min_kept"]

    SA_g = torch.empty_like(SA_e)
    x_g = torch.empty_like(x_e)
    res_g = torch.zeros_like(res_e)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st = torch.cuda.current_stream()
        S.apply(A, out=SA_g, ws=ws_a, stream=st)
        S.lstsq_solve_async(A, b, x_g, ws_s, result=res_g, stream=st)
    for rep in range(3):
        SA_g.fill_(float("nan"))
        x_g.fill_(float("nan"))
        res_g.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(SA_g, SA_e), "replay %d: SA differs" % rep
        assert torch.equal(x_g, x_e), "replay %d: x differs" % rep
        assert lib.read_solve_result(res_g) == (r_e, smax_e, smin_e)
        # eager work on the same buffers between replays
        S.apply(A, out=SA_g, ws=ws_a)
        torch.cuda.synchronize()
    del g


def test_async_solve_requires_workspace(lib):
    n, m = 5000, 8
    S = lib.Sketch("sparsestack", 32, n, 4, 3)
    A = torch.randn((n, m), dtype=torch.float64, device="cuda")
    b = torch.randn(n, dtype=torch.float64, device="cuda")
    x = torch.full((m,), 5.0, dtype=torch.float64, device="cuda")
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.SketchError):
        S.lstsq_solve_async(A, b, x, small)
    torch.cuda.synchronize()
    assert bool((x == 5.0).all())
