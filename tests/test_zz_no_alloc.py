"""GPU test of sketch_apply_noalloc, the allocation-free variant of
sketch_apply (its scratch lives in a fixed device array of the library),
through the C-ABI: on two calls in a row, the second with a smaller input,
its result is bitwise the result of sketch_apply with a workspace (the same
kernels in the same order); an input whose scratch exceeds the fixed size is
refused before any work, and an unsupported sketch kind is refused."""
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


def _case(lib, n, m, d, zeta, seed, dtype):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn((n, m), generator=g, dtype=torch.float64, device="cuda").to(dtype)
    S = lib.Sketch("sparsestack", d, n, zeta, seed)
    ws = torch.empty(S.workspace_size(0, dtype, m), dtype=torch.uint8, device="cuda")
    return S, A, ws


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_noalloc_matches_apply_on_two_calls(lib, dtype):
    # first call, then a smaller one (fewer rows and columns): the scratch
    # keeps the first call's contents, which must not leak into the second
    for n, m, d, zeta, seed in ((300001, 64, 256, 8, 3), (50021, 20, 96, 4, 4)):
        S, A, ws = _case(lib, n, m, d, zeta, seed, dtype)
        print("noalloc case n=%d m=%d d=%d zeta=%d dtype=%s" % (n, m, d, zeta, dtype), flush=True)
        ref = S.apply(A, ws=ws)
        got = S.apply_noalloc(A)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


def test_noalloc_refuses_too_large_and_other_kinds(lib):
    cap = lib.load().sketch_noalloc_scratch_bytes()
    n, m, d, zeta = 1 << 22, 200, 800, 8  # needs several hundred MB of scratch
    S = lib.Sketch("sparsestack", d, n, zeta, 1)
    need = S.workspace_size(0, torch.float64, m)
    assert need > cap
    A = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    out = torch.full((d, m), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SketchError) as e:
        S.apply_noalloc(A, out=out)
    assert e.value.code == lib.SK_E_NOTSUP and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    G = lib.Sketch("gaussian", 16, 1000, 1, 2)
    with pytest.raises(lib.SketchError):
        G.apply_noalloc(torch.zeros((1000, 8), dtype=torch.float64, device="cuda"))
